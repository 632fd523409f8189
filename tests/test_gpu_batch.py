"""GPU: batches of averaged right-hand-side problems on different meshes
(pa_batch_*), run concurrently or captured into one graph, against the same
problems evaluated one at a time, and against the oracle."""
import numpy as np
import pytest

from gpu_common import PARITY, bumps, check_parity, onodes, pair, rel_w, to_dev

pytestmark = pytest.mark.gpu

# (level, members): three meshes, different ensemble sizes
ITEMS = [(2, 3), (3, 2), (4, 1)]


def _problem(seed0=0):
    states, ops = [], []
    for i, (level, members) in enumerate(ITEMS):
        om, oo, lm, lo, mm, lb = pair(level)
        U = bumps(om, range(seed0 + 10 * i, seed0 + 10 * i + members))
        states.append(to_dev(mm.state(U)))
        ops.append(lo)
    return ops, states


def _singles(ops, avg, states, cfg):
    return [lo.phase_avg_rhs(avg, U, cfg)[0].cpu().numpy() for lo, U in zip(ops, states)]


CFGS = {
    "cg_polled": dict(solver=0, use_graph=False),
    "cg_graph": dict(solver=0, use_graph=True),
    "cheb_eager": dict(solver=1, use_graph=False),
    "cheb_graph": dict(solver=1, use_graph=True),
    "fp32_refined_graph": dict(solver=1, precision=1, use_graph=True),
}


@pytest.mark.parametrize("name", list(CFGS))
def test_gpu_batch_equals_single_calls(name):
    """Every item of a mixed-mesh batch equals the single-problem call with
    the same configuration bit for bit (same kernels, same launch shapes,
    deterministic reductions), on two calls in a row."""
    import torch
    from paper_2103_07706_amd import pa
    ops, states = _problem()
    avg = pa.Avg(8, 3600.0)
    kw = dict(CFGS[name])
    cfg = pa.solve_cfg(backward=pa.PA_BACKWARD_CLENSHAW, cg_rtol=1e-12, **kw)
    ref = _singles(ops, avg, states, cfg)
    b = pa.Batch(ops[0].ctx, list(zip(ops, [m for _, m in ITEMS])), avg)
    outs = [torch.full_like(U, float("nan")) for U in states]
    for rep in range(2):
        for o in outs:
            o.fill_(float("nan"))
        _, st = b.run(states, cfg, outs)
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, ref)):
            assert np.array_equal(o.cpu().numpy(), r), (name, rep, i)
        assert len(st) == len(ITEMS)
        if kw.get("use_graph") and rep == 1:
            assert all(s["graph"] == 1 for s in st)
        ops[0].swe_nonlinear(states[0])  # unrelated eager work between calls


def test_gpu_batch_parity_with_oracle():
    """Each item of a batch against the oracle, parity mode."""
    from paper_2103_07706_amd import pa
    avg = pa.Avg(8, 3600.0)
    cfg = pa.solve_cfg(backward=pa.PA_BACKWARD_CLENSHAW, weight_cut=0.0,
                       solver=pa.PA_SOLVER_CHEBYSHEV, use_graph=True, **PARITY)
    ops, states, refs = [], [], []
    for level, seed in [(2, 5), (3, 6)]:
        om, oo, lm, lo, mm, lb = pair(level)
        U = bumps(om, [seed])
        ops.append(lo)
        states.append(to_dev(mm.state(U)))
        refs.append((oo, mm, oo.phase_avg_rhs(lb, *onodes(avg), U[0], tol=1e-13, rtol=1e-14)))
    b = pa.Batch(ops[0].ctx, [(o, 1) for o in ops], avg)
    outs, st = b.run(states, cfg)
    for (oo, mm, ref), o in zip(refs, outs):
        got = mm.back(o.cpu().numpy())[0]
        check_parity(oo, got, ref, 1e-12)


def test_gpu_batch_autotune_and_replay(tmp_path):
    """Per-item launch shapes from the autotuner (stored in and reloaded from
    a JSON cache) keep every item within parity of the default shape, and the
    captured batch replays identically."""
    import torch
    from paper_2103_07706_amd import pa
    ops, states = _problem(seed0=3)
    avg = pa.Avg(8, 3600.0)
    cfg = pa.solve_cfg(backward=pa.PA_BACKWARD_CLENSHAW, cg_rtol=1e-12,
                       solver=pa.PA_SOLVER_CHEBYSHEV, use_graph=True)
    b = pa.Batch(ops[0].ctx, list(zip(ops, [m for _, m in ITEMS])), avg)
    ref, _ = b.run(states, cfg)
    ref = [r.cpu().numpy() for r in ref]
    before = pa.lib()
    keep = pa.LaunchTune()
    pa._check(before.pa_get_launch_tune(keep))
    cache = str(tmp_path / "batch_tune.json")
    tunes = b.autotune(states, cfg, cache=cache)
    assert len(tunes) == len(ITEMS) and not any(t["cached"] for t in tunes)
    after = pa.LaunchTune()
    pa._check(before.pa_get_launch_tune(after))
    assert (after.narrow_rows_per_thread, after.wide_max_wg) == \
        (keep.narrow_rows_per_thread, keep.wide_max_wg)  # process-wide shape untouched
    outs = [torch.empty_like(U) for U in states]
    first = None
    for rep in range(3):
        _, st = b.run(states, cfg, outs)
        got = [o.cpu().numpy() for o in outs]
        for g, r in zip(got, ref):
            assert np.abs(g - r).max() <= 1e-11 * np.abs(r).max()
        if first is None:
            first = got
        else:
            assert all(np.array_equal(a, c) for a, c in zip(first, got))
    b2 = pa.Batch(ops[0].ctx, list(zip(ops, [m for _, m in ITEMS])), avg)
    again = b2.autotune(states, cfg, cache=cache)
    assert all(t["cached"] for t in again)
    assert [b2.get_tune(i) for i in range(len(ITEMS))] == \
        [{k: t[k] for k in pa.TUNE_FIELDS} for t in tunes]


def test_gpu_batch_errors():
    """A workspace below the reported size is refused before any launch;
    states of the wrong shape are refused by the binding."""
    import ctypes

    import torch
    from paper_2103_07706_amd import pa
    ops, states = _problem()
    avg = pa.Avg(4, 1000.0)
    b = pa.Batch(ops[0].ctx, list(zip(ops, [m for _, m in ITEMS])), avg)
    cfg = pa.solve_cfg()
    ws, nb = b.workspace(cfg)
    outs = [torch.empty_like(U) for U in states]
    up, op = b._ptrs(states, outs)
    code = pa.lib().pa_batch_run(ops[0].ctx._h, b._h, up, op, ws, 1024, ctypes.byref(cfg), None)
    assert code == pa.PA_ENOMEM
    with pytest.raises(ValueError):
        b.run(states[::-1], cfg)
