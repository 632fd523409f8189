"""Pins for the oracle's mesh, operators, mass solve and spectral estimate.

Each test checks the oracle against something other than itself: the paper's
printed mesh statistics, closed forms (Euler characteristic, gravity-wave
frequency on the sphere), structural identities of the compatible pair, or a
library routine (scipy).
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from paper_2103_07706_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_kv(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                out[k] = float(v)
    return out


def _mats(ops):
    ex = ops.export()
    ne = ops.mesh.ne
    rows = np.repeat(np.arange(ne), np.diff(ex["rowptr"]))
    M = sp.coo_matrix((ex["mass"], (rows, ex["cols"])), shape=(ne, ne)).tocsr()
    F = sp.coo_matrix((ex["cor"], (rows, ex["cols"])), shape=(ne, ne)).tocsr()
    return M, F, ex["area"]


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_mesh_counts_and_euler(oracle_mesh, level):
    m = oracle_mesh(level)
    assert m.nc == 20 * 4 ** level
    assert m.ne == 30 * 4 ** level
    assert m.nv == 10 * 4 ** level + 2
    assert m.nv - m.ne + m.nc == 2
    # every edge has two distinct cells; every cell three distinct edges
    assert np.all(m.edge_cells[:, 0] < m.edge_cells[:, 1])
    assert np.all(np.sort(m.cell_edges, axis=1)[:, :-1] != np.sort(m.cell_edges, axis=1)[:, 1:])
    # vertices on the sphere
    np.testing.assert_allclose(np.linalg.norm(m.verts, axis=1), m.radius, rtol=1e-14)


def test_mesh_level5_matches_paper(oracle_mesh):
    g = _read_kv("mesh_level5.txt")
    m = oracle_mesh(int(g["level"]))
    assert m.nc == int(g["cells"])
    e = m.verts[m.edge_verts[:, 0]] - m.verts[m.edge_verts[:, 1]]
    lmax = np.linalg.norm(e, axis=1).max() / 1e3
    assert abs(lmax - g["max_distance_km"]) < 1.0


@pytest.mark.parametrize("level", [1, 3])
def test_mesh_orientation(oracle_mesh, level):
    m = oracle_mesh(level)
    P = m.verts[m.cell_verts]
    k = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    assert np.all(np.einsum("ij,ij->i", k, P.sum(axis=1)) > 0)  # CCW from outside
    # edge a->b runs CCW around c0: it is local side (v_{i+1}, v_{i+2}) of c0
    for e in range(0, m.ne, max(1, m.ne // 50)):
        c0 = m.edge_cells[e, 0]
        i = list(m.cell_edges[c0]).index(e)
        assert m.cell_verts[c0, (i + 1) % 3] == m.edge_verts[e, 0]
        assert m.cell_verts[c0, (i + 2) % 3] == m.edge_verts[e, 1]
        assert m.cell_sign[c0, i] == 1
        c1 = m.edge_cells[e, 1]
        assert m.cell_sign[c1, list(m.cell_edges[c1]).index(e)] == -1


@pytest.mark.parametrize("level", [1, 3])
def test_operator_structure(oracle_ops, level):
    """W L is skew (L purely oscillatory), M_u SPD, five entries per row."""
    o = oracle_ops(level)
    M, F, area = _mats(o)
    assert abs(M - M.T).max() == 0.0
    assert abs(F + F.T).max() <= 1e-15 * abs(F).max()
    assert np.all(np.diff(o.export()["rowptr"]) == 5)
    assert np.all(M.diagonal() > 0)
    w = np.linalg.eigvalsh(M.toarray()) if level == 1 else None
    if w is not None:
        assert w.min() > 0
    # total area of the polyhedron is below the sphere's and close to it
    S = 4 * np.pi * o.mesh.radius ** 2
    assert area.sum() < S and area.sum() > (0.9 if level == 1 else 0.99) * S


def test_dense_spectrum_imaginary(oracle_ops):
    o = oracle_ops(1)
    n = o.n
    Ld = np.column_stack([o.apply_L(np.eye(n)[j]) for j in range(n)])
    ev = np.linalg.eigvals(Ld)
    rho = np.abs(ev).max()
    assert np.abs(ev.real).max() <= 1e-12 * rho


def test_gravity_wave_frequency_converges(oracle_ops):
    """With Omega = 0 the slowest gravity waves have omega^2 = 2 g H / R^2
    (spherical harmonic degree 1)."""
    exact = np.sqrt(2 * 9.80616 * 1000.0) / 6.37122e6
    errs = []
    for level in (1, 2):
        o = oracle_ops(level, Omega=0.0)
        n = o.n
        Ld = np.column_stack([o.apply_L(np.eye(n)[j]) for j in range(n)])
        w = np.abs(np.linalg.eigvals(Ld))
        w = np.sort(w[w > 1e-3 * exact])
        errs.append(abs(w[0] - exact) / exact)
    assert errs[1] < errs[0] and errs[1] < 0.03


def test_linear_geostrophic_balance_converges(oracle_mesh, oracle_ops):
    """Small-amplitude zonal flow: f u^perp + g grad eta -> 0 (signs and
    scales of Coriolis and pressure gradient against each other)."""
    ph = inputs.Physics(H=5960.0)
    rel = []
    for level in (3, 4, 5):
        m = oracle_mesh(level)
        o = oracle_ops(level, H=5960.0)
        M, F, area = _mats(o)
        U = inputs.balanced_zonal_state(m.verts, m.cell_verts, m.edge_verts, u0=0.01, phys=ph)
        u, eta = U[:m.ne], U[m.ne:]
        Dt = np.zeros(m.ne)
        for i in range(3):
            np.add.at(Dt, m.cell_edges[:, i], m.cell_sign[:, i] * eta)
        a = -(F @ u)
        rel.append(np.linalg.norm(a + o.g * Dt) / np.linalg.norm(a))
    assert rel[0] < 0.02 and rel[1] < rel[0] / 2.5 and rel[2] < rel[1] / 2.5


def test_mass_matrix_energy_converges(oracle_mesh, oracle_ops):
    """u'M u of the RT0 field of a solid-body rotation tends to the integral
    of |u|^2 over the sphere, omega^2 (8 pi / 3) R^4."""
    R = 6.37122e6
    u0 = 20.0
    exact = (u0 / R) ** 2 * 8 * np.pi / 3 * R ** 4
    errs = []
    for level in (2, 3, 4):
        m = oracle_mesh(level)
        M, _, _ = _mats(oracle_ops(level))
        U = inputs.balanced_zonal_state(m.verts, m.cell_verts, m.edge_verts, u0=u0)
        u = U[:m.ne]
        errs.append(abs(u @ (M @ u) - exact) / exact)
    assert errs[2] < 0.01 and errs[2] < errs[1] < errs[0]


def test_divergence_sums_to_zero(oracle_mesh):
    """1' D = 0: each edge enters its two cells with opposite signs."""
    m = oracle_mesh(3)
    col = np.zeros(m.ne)
    for i in range(3):
        np.add.at(col, m.cell_edges[:, i], m.cell_sign[:, i])
    assert np.all(col == 0)


def test_mass_solve_matches_scipy(oracle_ops):
    o = oracle_ops(3)
    M, _, _ = _mats(o)
    b = np.random.default_rng(3).standard_normal(o.mesh.ne)
    x, it = o.mass_solve(b, rtol=1e-14)
    ref = spla.spsolve(M.tocsc(), b)
    assert np.linalg.norm(x - ref) <= 1e-13 * np.linalg.norm(ref)
    assert it < 30
    assert np.linalg.norm(M @ x - b) <= 1e-14 * np.linalg.norm(b) * 1.01


def test_mass_solve_iterations_mesh_independent(oracle_ops):
    """Sec. 2.5: the velocity solve converges in a mesh-independent number
    of iterations."""
    its = []
    for level in (2, 3, 4, 5):
        o = oracle_ops(level)
        b = np.random.default_rng(level).standard_normal(o.mesh.ne)
        its.append(o.mass_solve(b, rtol=1e-10)[1])
    assert max(its) - min(its) <= 3 and max(its) <= 20


def test_power_estimate_bounds_spectral_radius(oracle_ops):
    for level in (1, 2):
        o = oracle_ops(level)
        n = o.n
        Ld = np.column_stack([o.apply_L(np.eye(n)[j]) for j in range(n)])
        rho = np.abs(np.linalg.eigvals(Ld)).max()
        lb = oracle.lambda_bar(o, iters=300)
        assert 1.0 <= lb / rho <= 1.1
