"""Pins for the oracle's rational (REXI) exponential (Sec. 2.4 and Sec. 4:
the exponential as a sum of rational functions of L whose terms are
independent shifted solves).

Against: the closed form exp(i theta x) itself (the rational function of the
trapezoidal rule on the ellipse must reproduce it on [-1, 1] to the
quadrature's geometric accuracy, and exactly in the limit of a constant),
a dense matrix exponential (scipy expm) in the energy-scaled coordinates
where L is skew, the oracle's Chebyshev exponential (a different
construction of the same function of L), and the invariants of exp(tL)
(energy, inverse, the group property).  A dropped Jacobian factor sinh, a
flipped sign of theta, nodes without the half-step offset or a missing real
part fail these tests.
"""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from paper_2103_07706_amd import inputs
from test_oracle_exponential import _dense

# (theta, N, eta0) with the rational function within 1e-12 of exp(i theta x)
CASES = [(1.0, 24, 1.29), (5.41, 36, 0.79), (-5.41, 36, 0.79), (11.0, 48, 0.60)]


def _r(theta, N, eta0, x):
    X, c = oracle.rexi_coeffs(theta, N, eta0)
    return (c[None, :] / (X[None, :] - x[:, None])).sum(axis=1)


@pytest.mark.parametrize("theta,N,eta0", CASES)
def test_rational_function_reproduces_exponential(theta, N, eta0):
    x = np.cos(np.pi * np.arange(4001) / 4000)
    err = np.abs(_r(theta, N, eta0, x) - np.exp(1j * theta * x)).max()
    assert err < 2e-12, err
    # fewer nodes on the same ellipse: geometric loss of accuracy
    err_half = np.abs(_r(theta, N // 2, eta0, x) - np.exp(1j * theta * x)).max()
    assert err_half > 100 * err


def test_rational_function_of_a_constant():
    """theta = 0: the Cauchy integral of 1/(X - x) over the ellipse is 1; the
    trapezoidal rule reaches it geometrically, like exp(-N eta0)."""
    x = np.linspace(-1, 1, 501)
    assert np.abs(_r(0.0, 48, 1.0, x) - 1.0).max() < 1e-14
    e24 = np.abs(_r(0.0, 24, 1.0, x) - 1.0).max()
    assert 1e-12 < e24 < 1e-9


def test_nodes_come_in_conjugate_pairs():
    """z_j = i theta X_j: the nodes phi and pi - phi give conjugate z and
    conjugate terms i theta c_j (the real sum of the real operator)."""
    theta, N, eta0 = 5.41, 36, 0.79
    X, c = oracle.rexi_coeffs(theta, N, eta0)
    z, w = 1j * theta * X, 1j * theta * c
    for j in range(N):
        k = (N // 2 - 1 - j) % N
        assert abs(z[k] - np.conj(z[j])) < 1e-12 * abs(z[j])
        assert abs(w[k] - np.conj(w[j])) < 1e-12 * abs(w).max()


@pytest.fixture(scope="module")
def level1(oracle_mesh, oracle_ops):
    m = oracle_mesh(1)
    o = oracle_ops(1)
    Ld, W, Wh, Whi = _dense(o)
    lb = oracle.lambda_bar(o, iters=300)
    U = inputs.gaussian_bumps_state(m.verts, m.cell_verts, m.edge_verts, 10, 0)
    return o, Ld, W, Wh, Whi, lb, U


@pytest.mark.parametrize("t", [600.0, -1800.0, 7200.0])
def test_rexi_matches_dense_expm(level1, t):
    o, Ld, W, Wh, Whi, lb, U = level1
    S = Wh @ Ld @ Whi
    ref = Whi @ sl.expm(t * S) @ (Wh @ U)
    theta = lb * t
    N, eta0 = (24, 1.29) if abs(theta) <= 1.0 else (36, 0.79)
    assert abs(theta) <= 5.41
    out, it = o.rexi_expL(lb, t, U, N, eta0, gm_rtol=1e-14, rtol=1e-15)
    wn = lambda X: np.sqrt(X @ W @ X)
    assert wn(out - ref) <= 1e-11 * wn(U), wn(out - ref) / wn(U)
    assert it > 0


def test_rexi_matches_chebyshev_and_invariants(oracle_mesh, oracle_ops):
    m = oracle_mesh(3)
    o = oracle_ops(3)
    lb = oracle.lambda_bar(o, iters=200)
    U = inputs.gaussian_bumps_state(m.verts, m.cell_verts, m.edge_verts, 10, 0)
    t = 3600.0
    assert lb * t <= 5.41
    E, _ = o.rexi_expL(lb, t, U, 36, 0.79)
    C, _ = o.expL(lb, t, U, tol=1e-13, rtol=1e-14)
    assert o.wnorm(E - C) <= 1e-11 * o.wnorm(U)
    assert abs(o.wnorm(E) / o.wnorm(U) - 1) <= 1e-11
    # inverse and group property
    Z, _ = o.rexi_expL(lb, -t, E, 36, 0.79)
    assert o.wnorm(Z - U) <= 1e-11 * o.wnorm(U)
    A, _ = o.rexi_expL(lb, 0.5 * t, U, 36, 0.79)
    B, _ = o.rexi_expL(lb, 0.5 * t, A, 36, 0.79)
    assert o.wnorm(B - E) <= 1e-11 * o.wnorm(U)


def _level(oracle_mesh, oracle_ops, level):
    m = oracle_mesh(level)
    o = oracle_ops(level)
    lb = oracle.lambda_bar(o, iters=200)
    U = inputs.gaussian_bumps_state(m.verts, m.cell_verts, m.edge_verts, 10, 0)
    return m, o, lb, U


def test_rexi_average_matches_chebyshev_average(oracle_mesh, oracle_ops):
    """Nbar with REXI exponentials against Nbar with Chebyshev exponentials
    (the same averaged operator, Sec. 2.2, by two constructions of exp(sL))."""
    m, o, lb, U = _level(oracle_mesh, oracle_ops, 2)
    s, w = oracle.avg_nodes(8, 3600.0)
    assert lb * 1800.0 <= 5.41
    R = o.rexi_phase_avg_rhs(lb, s, w, U, 36, 0.79, gm_rtol=1e-14, rtol=1e-15)
    C = o.phase_avg_rhs(lb, s, w, U, tol=1e-14, rtol=1e-15)
    assert o.wnorm(R - C) <= 1e-10 * o.wnorm(C), o.wnorm(R - C) / o.wnorm(C)
    # with the identity in place of N the average is U itself (sum w = 1 and
    # exp(-sL) exp(sL) = I up to the rational approximation); level 1
    m, o, lb, U = _level(oracle_mesh, oracle_ops, 1)
    I = o.rexi_phase_avg_rhs(lb, s, w, U, 36, 0.79, gm_rtol=1e-14, rtol=1e-15, which=1)
    assert o.wnorm(I - U) <= 1e-11 * o.wnorm(U)
    # with L in place of N: L U (the group property and sum w = 1)
    LU = o.apply_L(U, rtol=1e-15)
    A = o.rexi_phase_avg_rhs(lb, s, w, U, 36, 0.79, gm_rtol=1e-14, rtol=1e-15, which=2)
    assert o.wnorm(A - LU) <= 1e-10 * o.wnorm(LU)


def test_rexi_step_matches_chebyshev_step(oracle_mesh, oracle_ops):
    m, o, lb, U = _level(oracle_mesh, oracle_ops, 1)
    s, w = oracle.avg_nodes(8, 3600.0)
    R = o.rexi_step(lb, s, w, 1800.0, U, 36, 0.79, gm_rtol=1e-14, rtol=1e-15)
    C = o.step(lb, s, w, 1800.0, U, tol=1e-14, rtol=1e-15)
    assert o.wnorm(R - C) <= 1e-10 * o.wnorm(U), o.wnorm(R - C) / o.wnorm(U)
    assert o.wnorm(R - U) > 1e-3 * o.wnorm(U)  # the step moved the state
