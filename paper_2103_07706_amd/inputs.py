"""Seeded synthetic inputs for the phase-averaged shallow-water path.

This module holds no arithmetic of the method itself: it only draws seeded
random numbers and evaluates the closed-form initial fields that the
workloads are defined by, on mesh geometry handed in by the caller (either
the GPU library's mesh or any other mesh with the same arrays).  Tests and
the benchmark use it on both sides of a comparison.

Workload recipe (the paper evaluates on Williamson test case 5, Sec. 3; the
workloads here replace it with seeded Gaussian bumps on the same mesh family):

* per member, a SplitMix64 stream seeded with the member index draws, for
  each bump in turn, an amplitude a ~ U(20, 100) m, z ~ U(-1, 1) and a
  longitude ~ U(0, 2 pi) (area-uniform centres);
* eta(cell) = sum_b a_b exp(-(d_b / w)^2), w = 1000 km, d_b the great-circle
  distance from the bump centre to the radially projected cell centroid;
* velocity from a stream function at the vertices,
  psi(v) = sum_b (g / f_b) a_b exp(-(d_b(v) / w)^2), with the per-bump f-plane
  value f_b = 2 Omega sign(z_b) max(|z_b|, sin 10 deg) (sign(0) = +1), so that
  each bump is in geostrophic balance; the flux through an edge whose
  endpoints run a -> b counter-clockwise around the edge's first cell is
  psi(a) - psi(b) (u = k x grad psi), which is exactly divergence free.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) with uniform doubles
    taken from the top 53 bits."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / (1 << 53)))


@dataclass
class Physics:
    radius: float = 6.37122e6
    omega: float = 7.292e-5
    g: float = 9.80616
    H: float = 1000.0


def bump_params(seed: int, nbumps: int):
    """Amplitudes [nb], unit centre vectors [nb, 3] and centre z [nb]."""
    rng = SplitMix64(seed)
    amp = np.zeros(nbumps)
    cen = np.zeros((nbumps, 3))
    zc = np.zeros(nbumps)
    for b in range(nbumps):
        amp[b] = rng.uniform(20.0, 100.0)
        z = rng.uniform(-1.0, 1.0)
        lon = rng.uniform(0.0, 2.0 * math.pi)
        r = math.sqrt(max(0.0, 1.0 - z * z))
        cen[b] = (r * math.cos(lon), r * math.sin(lon), z)
        zc[b] = z
    return amp, cen, zc


def _bump_sum(points, amp, cen, coef, radius, width):
    p = points / np.linalg.norm(points, axis=1, keepdims=True)
    out = np.zeros(len(points))
    for b in range(len(amp)):
        d = radius * np.arccos(np.clip(p @ cen[b], -1.0, 1.0))
        out += coef[b] * amp[b] * np.exp(-(d / width) ** 2)
    return out


def gaussian_bumps_state(verts, cell_verts, edge_verts, nbumps: int, seed: int,
                         phys: Physics = Physics(), width: float = 1.0e6):
    """State [u (edge fluxes) | eta (cells)] for one member."""
    verts = np.asarray(verts, dtype=np.float64)
    amp, cen, zc = bump_params(seed, nbumps)
    centroids = verts[np.asarray(cell_verts)].mean(axis=1)
    eta = _bump_sum(centroids, amp, cen, np.ones(nbumps), phys.radius, width)
    fmin = math.sin(math.radians(10.0))
    fb = np.array([2.0 * phys.omega * (1.0 if z >= 0 else -1.0) * max(abs(z), fmin)
                   for z in zc])
    psi = _bump_sum(verts, amp, cen, phys.g / fb, phys.radius, width)
    ev = np.asarray(edge_verts)
    u = psi[ev[:, 0]] - psi[ev[:, 1]]
    return np.concatenate([u, eta])


def p1dg_bumps_state(verts, cell_verts, ne: int, nbumps: int, seed: int,
                     phys: Physics = Physics(), width: float = 1.0e6):
    """State of the BDM2 x P1DG pair (unknowns 3 ne + 3 nc velocity, then 3
    per cell depth): the velocity at rest and, for each cell, the bump sum
    of gaussian_bumps_state at the cell's three vertices (radially projected)
    as the coefficients of the cell's barycentric coordinates -- the
    geostrophic adjustment problem of the same bumps."""
    verts = np.asarray(verts, dtype=np.float64)
    amp, cen, zc = bump_params(seed, nbumps)
    ev = _bump_sum(verts, amp, cen, np.ones(nbumps), phys.radius, width)
    cv = np.asarray(cell_verts)
    return np.concatenate([np.zeros(3 * ne + 3 * len(cv)), ev[cv].ravel()])


def _bdm2_velocity_from_stream(verts, tri, ev, psi):
    """BDM2 unknowns of u = k x grad psi_h, psi_h the continuous piecewise-
    linear interpolant of the vertex values psi (constant in each flat
    cell, divergence free, held exactly by BDM2): normal flux density
    (psi(a) - psi(b)) / |b - a| at all three points of each edge, moments
    u . e1, u . e2 and 0 in each cell (e1 from the cell's vertex 0 to 1,
    e2 = k x e1)."""
    flux = (psi[ev[:, 0]] - psi[ev[:, 1]]) / np.linalg.norm(verts[ev[:, 1]] - verts[ev[:, 0]], axis=1)
    P = verts[tri]
    k = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    twoA = np.linalg.norm(k, axis=1)
    k /= twoA[:, None]
    grad = sum(psi[tri[:, r], None] * np.cross(k, P[:, (r + 2) % 3] - P[:, (r + 1) % 3])
               for r in range(3)) / twoA[:, None]
    u = np.cross(k, grad)
    e1 = (P[:, 1] - P[:, 0]) / np.linalg.norm(P[:, 1] - P[:, 0], axis=1)[:, None]
    e2 = np.cross(k, e1)
    mom = np.stack([np.einsum("cd,cd->c", u, e1), np.einsum("cd,cd->c", u, e2),
                    np.zeros(len(tri))], 1)
    return np.concatenate([np.repeat(flux, 3), mom.ravel()])


def bdm2_bumps_state(verts, cell_verts, edge_cells, edge_verts, nbumps: int, seed: int,
                     phys: Physics = Physics(), width: float = 1.0e6):
    """The bumps of gaussian_bumps_state on the BDM2 x P1DG unknowns: the
    same stream function psi at the vertices, the velocity k x grad psi_h
    (_bdm2_velocity_from_stream); depth: the bump sum at each cell's
    vertices."""
    verts = np.asarray(verts, dtype=np.float64)
    tri = np.asarray(cell_verts)
    amp, cen, zc = bump_params(seed, nbumps)
    fmin = math.sin(math.radians(10.0))
    fb = np.array([2.0 * phys.omega * (1.0 if z >= 0 else -1.0) * max(abs(z), fmin)
                   for z in zc])
    psi = _bump_sum(verts, amp, cen, phys.g / fb, phys.radius, width)
    eta = _bump_sum(verts, amp, cen, np.ones(nbumps), phys.radius, width)
    return np.concatenate([_bdm2_velocity_from_stream(verts, tri, np.asarray(edge_verts), psi),
                           eta[tri].ravel()])


def williamson5_bdm2_state(verts, cell_verts, edge_cells, edge_verts, phys: Physics = None,
                           u0: float = 20.0):
    """The paper's test case (Sec. 3) on the BDM2 x P1DG unknowns: the zonal
    flow from its stream function psi = -u0 z (z radially projected) as
    k x grad psi_h, and the free surface of williamson5_state at each
    cell's vertices, -(R Omega u0 + u0^2/2) z^2 / (g R^2) (the bottom left
    out: williamson5_bottom_p1dg)."""
    phys = TC5_PHYSICS if phys is None else phys
    verts = np.asarray(verts, dtype=np.float64)
    tri = np.asarray(cell_verts)
    R = phys.radius
    z = R * verts[:, 2] / np.linalg.norm(verts, axis=1)
    psi = -u0 * z
    eta = -(R * phys.omega * u0 + 0.5 * u0 * u0) * z * z / (phys.g * R * R)
    return np.concatenate([_bdm2_velocity_from_stream(verts, tri, np.asarray(edge_verts), psi),
                           eta[tri].ravel()])


def random_state(nu: int, nh: int, seed: int, u_scale: float = 10.0,
                 eta_scale: float = 50.0):
    """Independent normal unknowns (numpy's PCG64 stream of the seed):
    velocity unknowns with standard deviation u_scale (m/s), then depth
    unknowns with eta_scale (m).  Excites the whole spectrum of L."""
    rng = np.random.default_rng(seed)
    return np.concatenate([u_scale * rng.standard_normal(nu),
                           eta_scale * rng.standard_normal(nh)])


def balanced_zonal_state(verts, cell_verts, edge_verts, u0: float = 20.0,
                         phys: Physics = Physics()):
    """Zonal flow in geostrophic balance from the paper's test case (Sec. 3)
    with a flat bottom: h = H - (R Omega u0 + u0^2/2) z^2 / (g R^2),
    u = (u0/R)(-y, x, 0).  eta = h - H at radially projected centroids; the
    velocity comes from its stream function psi = -u0 z, so fluxes are
    psi(a) - psi(b) along each edge.  An exact steady state of the continuous
    equations."""
    verts = np.asarray(verts, dtype=np.float64)
    R = phys.radius
    c = verts[np.asarray(cell_verts)].mean(axis=1)
    c = R * c / np.linalg.norm(c, axis=1, keepdims=True)
    eta = -(R * phys.omega * u0 + 0.5 * u0 * u0) * c[:, 2] ** 2 / (phys.g * R * R)
    vz = R * verts[:, 2] / np.linalg.norm(verts, axis=1)
    psi = -u0 * vz
    ev = np.asarray(edge_verts)
    u = psi[ev[:, 0]] - psi[ev[:, 1]]
    return np.concatenate([u, eta])


def williamson5_bottom(verts, cell_verts, b0: float = 2000.0, r0: float = math.pi / 9.0,
                       lat_c: float = math.pi / 6.0, lon_c: float = -math.pi / 2.0):
    """The isolated mountain of the paper's test case (Sec. 3): a cone of
    height b0 over the radius r0 in (latitude, longitude), centred at
    (lat_c, lon_c), at the radially projected cell centroids."""
    verts = np.asarray(verts, dtype=np.float64)
    c = verts[np.asarray(cell_verts)].mean(axis=1)
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    lat = np.arcsin(np.clip(c[:, 2], -1.0, 1.0))
    lon = np.arctan2(c[:, 1], c[:, 0])
    r = np.sqrt(np.minimum(r0 * r0, (lat - lat_c) ** 2 + (lon - lon_c) ** 2))
    return b0 * (1.0 - r / r0)


def williamson5_bottom_p1dg(verts, cell_verts, **kw):
    """The same mountain as P1DG coefficients: its height at each cell's
    three vertices (radially projected), cell by cell."""
    verts = np.asarray(verts, dtype=np.float64)
    at_v = williamson5_bottom(verts, np.repeat(np.arange(len(verts))[:, None], 3, axis=1), **kw)
    return at_v[np.asarray(cell_verts)].ravel()


def williamson5_state(verts, cell_verts, edge_verts, phys: Physics = None, u0: float = 20.0):
    """Initial state of the paper's test case (Sec. 3, flow over a mountain):
    the zonal flow u = (u0/R)(-y, x, 0) and the free surface in geostrophic
    balance with it, H + eta = H - (R Omega u0 + u0^2/2) z^2 / (g R^2), the
    bottom (williamson5_bottom) left out of eta (the layer depth is
    H + eta - b).  Physics: R = 6.37122e6 m, Omega = 7.292e-5 1/s, g = 9.8
    m/s^2, H = 5960 m (TC5_PHYSICS)."""
    return balanced_zonal_state(verts, cell_verts, edge_verts, u0=u0,
                                phys=TC5_PHYSICS if phys is None else phys)


TC5_PHYSICS = Physics(g=9.8, H=5960.0)


@dataclass
class Workload:
    """One synthetic workload: mesh level, members, bumps, averaging."""
    name: str
    level: int
    nbumps: int
    M: int
    T: float
    dt: float
    members: int = 1
    steps: int = 1
    phys: Physics = field(default_factory=Physics)


WORKLOADS = {
    # level 3, M=8, T=1 h, one 30-minute step
    "l3_m8": Workload("l3_m8", level=3, nbumps=10, M=8, T=3600.0, dt=1800.0),
    # level 5, M=32, T=2 h, dt=1 h, 24 steps
    "l5_m32": Workload("l5_m32", level=5, nbumps=40, M=32, T=7200.0, dt=3600.0, steps=24),
    # level 5, 64 members x M=64
    "l5_m64_x64": Workload("l5_m64_x64", level=5, nbumps=40, M=64, T=7200.0, dt=3600.0,
                           members=64),
    # level 6, M=64, T=2 h (the throughput workload)
    "l6_m64": Workload("l6_m64", level=6, nbumps=40, M=64, T=7200.0, dt=3600.0, steps=24),
    # level 7, M=64, T=2 h
    "l7_m64": Workload("l7_m64", level=7, nbumps=40, M=64, T=7200.0, dt=3600.0),
}

# Batches of meshes of uneven size: (level, members) items, M = 64, T = 2 h,
# 40 bumps, member seeds 0, 1, ... per item.
BATCHES = {
    "mixed_l4l5l6": [(4, 16), (5, 8), (6, 4)],
}
