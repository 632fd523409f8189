"""GPU: the allocation-free averaged right-hand side
(pa_phase_avg_rhs_noalloc, workspace in the library's static device
scratch) against the workspace entry point pa_phase_avg_rhs on the same
inputs, through the C ABI: bit-identical results on two calls in a row, the
second on a smaller problem (the scratch keeps the first call's contents);
the oracle bar on top; a problem whose workspace exceeds the scratch is
refused before anything is launched."""
import ctypes

import numpy as np
import pytest

from gpu_common import PARITY, bumps, check_parity, onodes, pair, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(lo, avg, U, cfg):
    """The entry point through the C ABI (the binding's argument types);
    returns the status code instead of raising."""
    from paper_2103_07706_amd import pa
    out = U.new_empty(U.shape)
    st = pa.Stats()
    code = pa.lib().pa_phase_avg_rhs_noalloc(lo.ctx._h, lo._h, avg._h, U.shape[0], pa._ptr(U),
                                             pa._ptr(out), ctypes.byref(cfg), ctypes.byref(st))
    return code, out, st.as_dict()


@pytest.mark.parametrize("solver", [0, 1])
def test_noalloc_equals_workspace_entry(solver):
    import torch
    from paper_2103_07706_amd import pa
    cases = [(3, [0, 1, 2], 8, 3600.0), (2, [5], 4, 1800.0)]  # the second is smaller
    for level, seeds, M, T in cases:
        om, oo, lm, lo, mm, lb = pair(level)
        U = bumps(om, seeds)
        Ud = to_dev(mm.state(U))
        avg = pa.Avg(M, T)
        cfg = pa.solve_cfg(solver=solver, weight_cut=0.0, use_graph=False, **PARITY)
        ref, _ = lo.phase_avg_rhs(avg, Ud, cfg)
        code, got, st = _noalloc(lo, avg, Ud, cfg)
        torch.cuda.synchronize()
        assert code == 0, pa.lib().pa_last_error().decode()
        assert st["terms"] == M * len(seeds) and st["graph"] == 0
        assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy()), (level, solver)
        o = oo.phase_avg_rhs(lb, *onodes(avg), U[0], tol=1e-13, rtol=1e-14)
        check_parity(oo, mm.back(got.cpu().numpy()[0]), o, 1e-12, what=(level, solver))


def test_noalloc_refuses_oversized_problem():
    from paper_2103_07706_amd import pa
    from gpu_common import _ctx
    lm = pa.Mesh(5)
    lo = pa.Ops(_ctx(), lm)
    lo.lambda_bar = 2 * pair(4)[5]
    U = to_dev(np.zeros((1, lo.n)))
    cfg = pa.solve_cfg(precision=pa.PA_FP32_REFINED)
    code, _, _ = _noalloc(lo, pa.Avg(64, 7200.0), U, cfg)
    assert code == pa.PA_ENOMEM
    assert "static scratch" in pa.lib().pa_last_error().decode()
