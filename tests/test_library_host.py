"""Host-side checks of the HIP library that need no GPU: the shared object
loads and exports every entry point of include/pa.h, and its independently
written mesh generator produces the oracle's mesh up to numbering."""
import os
import re

import numpy as np
import pytest

from matching import MeshMap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pa_[A-Za-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2103_07706_amd import pa
    L = pa.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(pa.EXPORTS)


@pytest.mark.parametrize("level", [0, 2, 4])
def test_library_mesh_matches_oracle(oracle_mesh, level):
    from paper_2103_07706_amd import pa
    lm = pa.Mesh(level)
    om = oracle_mesh(level)
    assert (lm.nv, lm.ne, lm.nc) == (om.nv, om.ne, om.nc)
    mm = MeshMap(om, lm)
    # same cells on both sides of every edge, up to the normal's direction
    for e in range(0, lm.ne, max(1, lm.ne // 200)):
        oc = set(mm.cell[lm.edge_cells[e]])
        assert oc == set(om.edge_cells[mm.edge[e]])
    np.testing.assert_allclose(np.sort(np.linalg.norm(lm.verts, axis=1)),
                               np.sort(np.linalg.norm(om.verts, axis=1)), rtol=1e-15)
    # c0 is the lower-numbered cell; a -> b runs counter-clockwise about c0
    P = lm.verts[lm.cell_verts]
    k = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    assert np.all(np.einsum("ij,ij->i", k, P.sum(axis=1)) > 0)
    assert np.all(lm.edge_cells[:, 0] < lm.edge_cells[:, 1])


def test_library_rejects_bad_arguments():
    from paper_2103_07706_amd import pa
    with pytest.raises(pa.PAError):
        pa.Mesh(12)
    with pytest.raises(pa.PAError):
        pa.Avg(0, 100.0)


def test_learned_preconditioner_parameters_host(tmp_path):
    """The library's initial parameters are the definition's (FP64 values of
    the reference rounded to FP32); save/load round-trips; only the built
    network shape is accepted."""
    import ctypes

    import numpy as np

    from oracle import lp_ref
    from paper_2103_07706_amd import pa
    lp = pa.LearnedPrecond(seed=42)
    assert lp.n_params == lp_ref.n_params()
    ref = lp_ref.init_params(42).astype(np.float32)
    assert np.array_equal(lp.params, ref)
    th = ref + np.float32(0.25)
    lp.params = th
    path = tmp_path / "net.bin"
    lp.save(path)
    lp2 = pa.LearnedPrecond(seed=1)
    lp2.load(path)
    assert np.array_equal(lp2.params, th)
    h = ctypes.c_void_p()
    assert pa.lib().pa_lp_create(2, 32, 0, ctypes.byref(h)) == pa.PA_ENOTSUP
    (tmp_path / "bad.bin").write_bytes(b"nonsense")
    with pytest.raises(pa.PAError):
        lp2.load(tmp_path / "bad.bin")


@pytest.mark.parametrize("M", [1, 5, 8, 32, 64])
@pytest.mark.parametrize("T", [1000.0, 3600.0, 7200.0])
def test_library_avg_nodes_match_oracle(M, T):
    """The library's averaging nodes and weights (host code of the HIP
    library) equal the oracle's, computed separately from the same reading
    of the averaging formula (midpoints of the support of rho(s/T),
    weights normalised to sum to one)."""
    import oracle
    from paper_2103_07706_amd import pa
    a = pa.Avg(M, T)
    s, w = oracle.avg_nodes(M, T)
    assert np.array_equal(a.s, s)
    assert np.abs(a.w - w).max() <= 1e-15 * np.abs(w).max()
    assert abs(a.w.sum() - 1.0) < 1e-14


def test_solve_cfg_defaults_and_layout():
    """The ctypes mirror of pa_solve_cfg matches the C layout: the library's
    defaults read back field by field (a shifted field would read garbage)."""
    from paper_2103_07706_amd import pa
    c = pa.solve_cfg()
    assert (c.precision, c.backward, c.maxit, c.growth_guard) == (pa.PA_FP64, pa.PA_BACKWARD_CLENSHAW,
                                                                  100, 0)
    assert (c.cg_rtol, c.cheb_tol, c.weight_cut, c.inner_rtol) == (1e-10, 1e-6, 1e-16, 1e-6)
    assert (c.use_graph, c.solver, c.precond) == (1, pa.PA_SOLVER_CHEBYSHEV, pa.PA_PRECOND_JACOBI)
    assert (c.exponential, c.rexi_nodes, c.rexi_eta0) == (pa.PA_EXP_CHEBYSHEV, 0, 0.0)


def _host_ops(level, lambda_bar):
    """Operators on the host only (pa_ops_create needs no device)."""
    import ctypes

    from paper_2103_07706_amd import pa
    m = pa.Mesh(level)
    ph = pa.Phys(9.80616, 1000.0, 7.292e-5, None, lambda_bar)
    h = ctypes.c_void_p()
    assert pa.lib().pa_ops_create(m._h, ctypes.byref(ph), ctypes.byref(h)) == pa.PA_OK
    return m, h


def test_rexi_workspace_sizing_host():
    """Planning of the rational exponential on the host: the library picks
    a node set for the call's largest time (sizing runs the same planning
    code as the call), honours an explicit one, and refuses node counts
    that are not multiples of 4 or an ellipse parameter out of range."""
    import ctypes

    from paper_2103_07706_amd import pa
    m, h = _host_ops(3, 7.2e-4)
    try:
        avg = pa.Avg(8, 3600.0)
        sz = ctypes.c_size_t()
        cheb = pa.solve_cfg()
        assert pa.lib().pa_workspace_size(h, avg._h, 1, ctypes.byref(cheb), ctypes.byref(sz)) == 0
        auto = pa.solve_cfg(exponential=pa.PA_EXP_REXI)
        assert pa.lib().pa_workspace_size(h, avg._h, 2, ctypes.byref(auto), ctypes.byref(sz)) == 0
        assert sz.value > 0
        fixed = pa.solve_cfg(exponential=pa.PA_EXP_REXI, rexi_nodes=36, rexi_eta0=0.79)
        assert pa.lib().pa_workspace_size(h, avg._h, 1, ctypes.byref(fixed), ctypes.byref(sz)) == 0
        # 18 poles a member: 32 complex columns, eight blocks of them at level 3
        assert sz.value > 8 * 32 * 16 * (1920 + 1280)
        for N, eta0 in [(30, 0.79), (4, 0.79), (260, 0.5), (36, 0.0), (36, 3.5)]:
            bad = pa.solve_cfg(exponential=pa.PA_EXP_REXI, rexi_nodes=N, rexi_eta0=eta0)
            assert pa.lib().pa_workspace_size(h, avg._h, 1, ctypes.byref(bad),
                                              ctypes.byref(sz)) == pa.PA_EINVAL, (N, eta0)
        bad = pa.solve_cfg(exponential=7)
        assert pa.lib().pa_workspace_size(h, avg._h, 1, ctypes.byref(bad),
                                          ctypes.byref(sz)) == pa.PA_EINVAL
    finally:
        pa.lib().pa_ops_destroy(h)
