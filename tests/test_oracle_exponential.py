"""Pins for the oracle's Chebyshev exponential (paper Sec. 2.4).

Against: the Jacobi-Anger closed form of the coefficients (scipy's Bessel
functions), the paper's Table 1 for the truncation rule, a dense matrix
exponential (scipy expm) in the energy-scaled coordinates where L is skew,
and exact invariants of exp(tL): energy, mass and the group property.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp
import scipy.special as ss

import oracle
from paper_2103_07706_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("Lbar", [0.3, 4.0, 17.5, 45.0])
def test_coefficients_match_jacobi_anger(Lbar):
    """exp(i Lbar x) = sum_k (2 - delta_k0) i^k J_k(Lbar) T_k(x)."""
    npts = 2 * int(np.ceil(Lbar)) + 64
    a = oracle.cheb_coeffs(Lbar, npts)
    k = np.arange(npts + 1)
    ref = np.where(k == 0, 1.0, 2.0) * (1j ** k) * ss.jv(k, Lbar)
    assert np.abs(a - ref).max() < 2e-14


def _K(theta, tol=1e-6):
    a = oracle.cheb_coeffs(theta, 2 * int(np.ceil(theta)) + 64)
    return oracle.cheb_truncate(a, tol)


def _interval(count, scale):
    """theta interval on which K(scale*theta) - 1 == count (K is monotone)."""
    def first_at_least(c):
        lo, hi = 0.0, 200.0
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if _K(scale * mid) - 1 >= c:
                hi = mid
            else:
                lo = mid
        return hi
    return first_at_least(count), first_at_least(count + 1)


def test_truncation_rule_reproduces_table1():
    """Table 1: iteration counts at Delta s = 15/30/60 min for levels 3-5.
    With theta proportional to Delta s, the rule 'drop from the top while the
    dropped total magnitude stays <= 1e-6' and 'iterations = degree - 1'
    (recurrence steps after P_0 and P_1) must fit each row with one theta."""
    rows = np.loadtxt(os.path.join(GOLDEN, "table1_chebyshev_iterations.txt"), dtype=int)
    for level, c15, c30, c60 in rows:
        lo = hi = None
        for c, scale in ((c15, 1.0), (c30, 2.0), (c60, 4.0)):
            a, b = _interval(c, scale)
            lo = a if lo is None else max(lo, a)
            hi = b if hi is None else min(hi, b)
        assert lo < hi, f"level {level}: no common theta"
        th = 0.5 * (lo + hi)
        assert [_K(th) - 1, _K(2 * th) - 1, _K(4 * th) - 1] == [c15, c30, c60]


def test_truncated_tail_within_threshold():
    for theta in (0.5, 6.0, 30.0):
        a = oracle.cheb_coeffs(theta, 2 * int(np.ceil(theta)) + 64)
        for tol in (1e-6, 1e-10):
            K = oracle.cheb_truncate(a, tol)
            assert np.abs(a[K + 1:]).sum() <= tol
            assert np.abs(a[K:]).sum() > tol


def _dense(o):
    ex = o.export()
    ne = o.mesh.ne
    rows = np.repeat(np.arange(ne), np.diff(ex["rowptr"]))
    M = sp.coo_matrix((ex["mass"], (rows, ex["cols"])), shape=(ne, ne)).toarray()
    n = o.n
    Ld = np.column_stack([o.apply_L(np.eye(n)[j]) for j in range(n)])
    W = sl.block_diag(o.H * M, o.g * np.diag(ex["area"]))
    Wh = np.real(sl.sqrtm(W))
    return Ld, W, Wh, np.linalg.inv(Wh)


@pytest.fixture(scope="module")
def level1(oracle_mesh, oracle_ops):
    m = oracle_mesh(1)
    o = oracle_ops(1)
    Ld, W, Wh, Whi = _dense(o)
    lb = oracle.lambda_bar(o, iters=300)
    U = inputs.gaussian_bumps_state(m.verts, m.cell_verts, m.edge_verts, 10, 0)
    return o, Ld, W, Wh, Whi, lb, U


@pytest.mark.parametrize("t", [600.0, -1800.0, 3600.0, 7200.0])
def test_exponential_matches_dense_expm(level1, t):
    """Against scipy expm of S = W^1/2 L W^-1/2 (skew), mapped back: raw
    coordinates are badly scaled (||L||_2 >> rho(L)), so compare in the
    energy norm."""
    o, Ld, W, Wh, Whi, lb, U = level1
    S = Wh @ Ld @ Whi
    ref = Whi @ sl.expm(t * S) @ (Wh @ U)
    out, K = o.expL(lb, t, U, tol=1e-13, rtol=1e-15)
    wn = lambda X: np.sqrt(X @ W @ X)
    assert wn(out - ref) <= 1e-13 * wn(U)
    out6, K6 = o.expL(lb, t, U, tol=1e-6, rtol=1e-10)
    assert K6 < K
    assert wn(out6 - ref) <= 1e-5 * wn(U)


def test_exponential_invariants(oracle_mesh, oracle_ops):
    m = oracle_mesh(3)
    o = oracle_ops(3)
    lb = oracle.lambda_bar(o, iters=200)
    U = inputs.gaussian_bumps_state(m.verts, m.cell_verts, m.edge_verts, 10, 0)
    V = inputs.gaussian_bumps_state(m.verts, m.cell_verts, m.edge_verts, 10, 1)
    tol = 1e-13
    E, K = o.expL(lb, 2400.0, U, tol=tol)
    # energy (W-norm) preserved up to the truncation threshold
    assert abs(o.wnorm(E) / o.wnorm(U) - 1) <= 10 * tol
    # mass: L leaves the total mass unchanged, so only p(0) - 1 <= tol enters
    mU, mE = o.diagnostics(U)["mass"], o.diagnostics(E)["mass"]
    assert abs(mE / mU - 1) <= 10 * tol
    # group property
    A, _ = o.expL(lb, 1000.0, U, tol=tol)
    B, _ = o.expL(lb, 1400.0, A, tol=tol)
    assert o.wnorm(B - E) <= 1e-12 * o.wnorm(U)
    # inverse
    Z, _ = o.expL(lb, -2400.0, E, tol=tol)
    assert o.wnorm(Z - U) <= 1e-12 * o.wnorm(U)
    # linearity
    EV, _ = o.expL(lb, 2400.0, V, tol=tol)
    EUV, _ = o.expL(lb, 2400.0, 2.0 * U - 3.0 * V, tol=tol)
    assert o.wnorm(EUV - (2 * E - 3 * EV)) <= 1e-12 * o.wnorm(EUV)
    # t = 0 is the identity
    I0, K0 = o.expL(lb, 0.0, U)
    assert K0 == 0 and np.array_equal(I0, U)


def test_degree_grows_linearly_with_time(oracle_ops):
    """Table 1's remark: degree roughly linear in resolution and time."""
    o = oracle_ops(3)
    lb = oracle.lambda_bar(o, iters=200)
    Ks = [_K(lb * t) for t in (1800.0, 3600.0, 7200.0, 14400.0)]
    d = np.diff(Ks)
    assert np.all(d > 0) and d[-1] < 2.5 * d[-2]
