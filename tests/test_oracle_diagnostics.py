"""Pins for the oracle's diagnostics (the mass and energy of the test case,
Sec. 3): each quantity converges under refinement to a closed-form integral
over the sphere, at second order (errors shrink about four times a level).

* L2 norm and mass of eta = (z/R)^2: int (z/R)^4 dA = 4 pi R^2 / 5,
  int (z/R)^2 dA = 4 pi R^2 / 3.
* H(div) norm of the flux interpolant of grad_s z on the unit sphere, split
  into its two parts through the linear energy (eta = 0, H = 1 gives
  u'M u = 2 E_lin): int |grad_s z|^2 = 8 pi / 3 and, z being a degree-one
  spherical harmonic (Laplacian -2 z), int (div u)^2 = 16 pi / 3.
* Nonlinear energy of the balanced zonal flow of Sec. 3 over a bottom
  b = beta (z/R)^2: eta = -A (z/R)^2 with A = (R Omega u0 + u0^2/2)/g,
  |u|^2 = u0^2 (1 - (z/R)^2), so with int f(z) dA = 2 pi R^2 int_{-1}^{1}
  f(R x) dx the energy int (H + eta - b)|u|^2/2 + g eta^2/2 is
  pi R^2 u0^2 (4H/3 - 4(A + beta)/15) + 2 pi R^2 g A^2 / 5.

Dropping the area from the divergence term, or the depth perturbation from
the kinetic-energy weight, fails these tests."""
import numpy as np

import oracle
from paper_2103_07706_amd import inputs

LEVELS = (3, 4, 5)


def _second_order(errs, last):
    errs = [abs(e) for e in errs]
    assert errs[-1] < last, errs
    for a, b in zip(errs, errs[1:]):
        assert b < a / 3.0, errs


def _unit_centroids(m):
    c = m.verts[m.cell_verts].mean(axis=1)
    return c / np.linalg.norm(c, axis=1, keepdims=True)


def _grad_z_flux(m):
    """Edge fluxes of grad_s z = e_z - z x/|x|^2: two-point Gauss rule of its
    normal component along each flat edge (normal in the plane of the edge's
    first cell, pointing out of it)."""
    a = m.verts[m.edge_verts[:, 0]]
    b = m.verts[m.edge_verts[:, 1]]
    P = m.verts[m.cell_verts[m.edge_cells[:, 0]]]
    k = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    k /= np.linalg.norm(k, axis=1, keepdims=True)
    t = b - a
    ln = np.linalg.norm(t, axis=1)
    n = np.cross(t / ln[:, None], k)
    W = np.zeros(m.ne)
    g = 0.5 / np.sqrt(3.0)
    for xi in (0.5 - g, 0.5 + g):
        x = a + xi * (b - a)
        grad = -(x[:, 2] / np.einsum("ij,ij->i", x, x))[:, None] * x
        grad[:, 2] += 1.0
        W += 0.5 * ln * np.einsum("ij,ij->i", grad, n)
    return W


def test_l2_norm_and_mass_converge():
    R = 6.37122e6
    e_l2, e_mass = [], []
    for level in LEVELS:
        m = oracle.Mesh(level, radius=R)
        o = oracle.Ops(m)
        eta = _unit_centroids(m)[:, 2] ** 2
        d = o.diagnostics(np.concatenate([np.zeros(m.ne), eta]))
        e_l2.append(d["l2_eta"] / np.sqrt(4 * np.pi * R * R / 5) - 1)
        e_mass.append(d["mass"] / (4 * np.pi * R * R / 3) - 1)
    _second_order(e_l2, 3e-4)
    _second_order(e_mass, 6e-4)


def test_hdiv_norm_parts_converge():
    e_u, e_div = [], []
    for level in LEVELS:
        m = oracle.Mesh(level, radius=1.0)
        o = oracle.Ops(m, g=1.0, H=1.0, Omega=0.0)
        d = o.diagnostics(np.concatenate([_grad_z_flux(m), np.zeros(m.nc)]))
        uMu = 2.0 * d["energy_linear"]
        div2 = d["hdiv_u"] ** 2 - uMu
        e_u.append(uMu / (8 * np.pi / 3) - 1)
        e_div.append(div2 / (16 * np.pi / 3) - 1)
    _second_order(e_u, 1e-3)
    _second_order(e_div, 1.5e-4)


def test_nonlinear_energy_of_zonal_flow_converges():
    ph = inputs.Physics(H=5960.0)
    R, u0, beta = ph.radius, 20.0, 500.0
    A = (R * ph.omega * u0 + 0.5 * u0 * u0) / ph.g
    exact = (np.pi * R * R * u0 * u0 * (4 * ph.H / 3 - 4 * (A + beta) / 15)
             + 2 * np.pi * R * R * ph.g * A * A / 5)
    errs = []
    for level in LEVELS:
        m = oracle.Mesh(level, radius=R)
        b = beta * _unit_centroids(m)[:, 2] ** 2
        o = oracle.Ops(m, g=ph.g, H=ph.H, Omega=ph.omega, b=b)
        U = inputs.balanced_zonal_state(m.verts, m.cell_verts, m.edge_verts, u0=u0, phys=ph)
        errs.append(o.diagnostics(U)["energy_nonlinear"] / exact - 1)
    _second_order(errs, 6e-4)
