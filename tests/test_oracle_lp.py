"""Pins of the learned-preconditioner reference (oracle/lp_ref.py) against
things other than itself: finite differences, dense linear algebra and the
closed-form matrix derivative, and the identity at initialisation."""
import functools

import numpy as np
import pytest


@functools.lru_cache(maxsize=None)
def _graph(level):
    import oracle
    from oracle import lp_ref
    om = oracle.Mesh(level)
    oo = oracle.Ops(om)
    return lp_ref.Graph(om, oo)


def _theta(seed, scale=0.3):
    from oracle import lp_ref
    rng = np.random.default_rng(seed)
    return lp_ref.init_params(seed) + scale * rng.standard_normal(lp_ref.n_params())


def test_param_layout():
    from oracle import lp_ref
    assert lp_ref.n_params() == 16098
    th = lp_ref.init_params(7)
    p = lp_ref.unpack(th)
    assert np.array_equal(lp_ref.pack(p), th)
    # Glorot bounds and the zero/identity heads
    for name, sh in lp_ref.param_shapes():
        if name.endswith(".W"):
            assert np.abs(p[name]).max() <= np.sqrt(6.0 / (sh[0] + sh[1]))
    assert not p["hd.w"].any() and not p["p2.w"].any() and not p["p2.b"].any()


def test_initial_network_is_jacobi():
    """Zero head weights: Ghat = I (softplus(log(e - 1)) = 1, beta = 0)."""
    from oracle import lp_ref
    g = _graph(1)
    _, gd, beta, goff = lp_ref.forward(lp_ref.init_params(3), g)
    assert np.allclose(gd, 1.0, rtol=0, atol=1e-15)
    assert not beta.any() and not goff.any()


def test_features_are_dimensionless_and_bounded():
    g = _graph(2)
    assert abs(g.Fe[:, 1].mean() - 1.0) < 1e-12   # length / mean length
    assert abs(g.Fc[:, 0].mean() - 1.0) < 1e-12   # area / mean area
    assert np.all(g.Fe[:, 0] > 0)
    assert np.all(np.abs(g.Fe[:, 3:8]) <= 1.0 + 1e-12)
    # equilateral-like cells: angles near 60 degrees
    assert abs(g.Fe[:, 4].mean() - 0.5) < 0.05
    # scaled mass matrix: unit diagonal, symmetric
    from oracle import lp_ref
    Mh = lp_ref.mhat_dense(g)
    assert np.allclose(np.diag(Mh), 1.0, atol=1e-14)
    assert np.abs(Mh - Mh.T).max() < 1e-15


def test_loss_equals_dense_frobenius_with_identity_probes():
    """With the columns of I as probes, L = |Ghat^T Mhat Ghat - I|_F^2 / n, and
    dL/dGhat = (4/n) Mhat Ghat (A - I) on the pattern (matrix calculus for
    the symmetric A = Ghat^T Mhat Ghat)."""
    from oracle import lp_ref
    g = _graph(1)
    _, gd, beta, goff = lp_ref.forward(_theta(11), g)
    n = g.ne
    L, dd, do = lp_ref.loss_and_ghat_grad(g, gd, goff, np.eye(n))
    G = lp_ref.ghat_dense(g, gd, goff)
    Mh = lp_ref.mhat_dense(g)
    A = G.T @ Mh @ G
    R = A - np.eye(n)
    assert abs(L - (R * R).sum() / n) <= 1e-12 * L
    D = 4.0 / n * Mh @ G @ R
    assert np.abs(dd - np.diag(D)).max() <= 1e-12 * np.abs(D).max()
    assert np.abs(do - D[g.pi, g.pj]).max() <= 1e-12 * np.abs(D).max()


@pytest.mark.parametrize("seed", [1, 2])
def test_gradient_matches_central_differences(seed):
    """Manual backpropagation against central differences of the loss, on
    parameter entries drawn from every tensor."""
    from oracle import lp_ref
    g = _graph(1)
    th = _theta(seed)
    rng = np.random.default_rng(100 + seed)
    Z = rng.choice([-1.0, 1.0], size=(g.ne, 4))
    L, grad = lp_ref.loss_grad(th, g, Z)
    gnorm = np.linalg.norm(grad)
    idx, off = [], 0
    for name, sh in lp_ref.param_shapes():
        n = int(np.prod(sh))
        idx += list(off + rng.choice(n, size=min(n, 3), replace=False))
        off += n
    h = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (lp_ref.loss_grad(tp, g, Z)[0] - lp_ref.loss_grad(tm, g, Z)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-7 * gnorm + 1e-6 * abs(grad[i]), (i, fd, grad[i])


def test_preconditioner_is_spd_and_descent_lowers_the_loss():
    """P = D^-1/2 Ghat Ghat^T D^-1/2 is positive on probes; a few gradient
    steps lower the loss (the gradient is a descent direction)."""
    from oracle import lp_ref
    g = _graph(1)
    th = _theta(5, scale=0.1)
    rng = np.random.default_rng(9)
    Z = rng.choice([-1.0, 1.0], size=(g.ne, 8))
    _, gd, beta, goff = lp_ref.forward(th, g)
    G = lp_ref.ghat_dense(g, gd, goff)
    Dm = np.diag(1.0 / np.sqrt(g.diag))
    P = Dm @ G @ G.T @ Dm
    assert np.all(np.einsum("ip,ij,jp->p", Z, P, Z) > 0)
    L0, gr = lp_ref.loss_grad(th, g, Z)
    L1, _ = lp_ref.loss_grad(th - 1e-3 * gr / np.linalg.norm(gr), g, Z)
    assert L1 < L0
