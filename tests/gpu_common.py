"""Shared set-up of the GPU parity tests: the same seeded inputs on the
oracle's mesh and on the library's mesh, mapped by geometry.

The oracle side never takes anything the library computed: its averaging
nodes and weights come from ``oracle.avg_nodes`` (``onodes``), its lambda_bar
from the oracle's power iteration (the value is then given to the library,
as both sides must use the same Chebyshev scale)."""
import functools

import numpy as np

from matching import MeshMap

PARITY = dict(cheb_tol=1e-13, cg_rtol=1e-14)


def rel_w(ops_oracle, a, b):
    return ops_oracle.wnorm(a - b) / ops_oracle.wnorm(b)


def block_max(ne, a, b):
    """Largest pointwise difference of each block (u, eta), relative to the
    block's largest reference value: (max_u, max_eta).  A block whose
    reference is exactly zero is compared absolutely."""
    out = []
    for sl in (slice(0, ne), slice(ne, None)):
        d = np.abs(a[..., sl] - b[..., sl]).max()
        r = np.abs(b[..., sl]).max()
        out.append(d / r if r > 0 else d)
    return tuple(out)


def check_parity(oo, got, ref, tol, tol_max=None, what=""):
    """The parity bar: relative energy-norm difference below `tol` and the
    per-block relative max-norm differences below `tol_max` (default 10 tol:
    a single row may carry more of the difference than the norm shows).
    Returns (w, max_u, max_eta)."""
    tol_max = 10 * tol if tol_max is None else tol_max
    w = rel_w(oo, got, ref)
    mu, me = block_max(oo.mesh.ne, got, ref)
    assert w < tol, (what, "energy norm", w)
    assert mu < tol_max, (what, "u max-norm", mu)
    assert me < tol_max, (what, "eta max-norm", me)
    return w, mu, me


def onodes(avg):
    """The oracle's own nodes and weights for a library averaging object
    made from (M, T)."""
    import oracle
    assert avg.T is not None, "explicit nodes: build them on the oracle side"
    return oracle.avg_nodes(avg.M, avg.T)


@functools.lru_cache(maxsize=None)
def pair(level, lambda_iters=200):
    """(oracle mesh, oracle ops, library mesh, library ops, map, lambda_bar)."""
    import oracle
    from paper_2103_07706_amd import pa
    ctx = _ctx()
    om = oracle.Mesh(level)
    oo = oracle.Ops(om)
    lm = pa.Mesh(level)
    lo = pa.Ops(ctx, lm)
    lb = oracle.lambda_bar(oo, iters=lambda_iters)
    lo.lambda_bar = lb
    return om, oo, lm, lo, MeshMap(om, lm), lb


@functools.lru_cache(maxsize=None)
def _ctx():
    from paper_2103_07706_amd import pa
    return pa.Context(0)


def bumps(om, seeds, nb=10):
    from paper_2103_07706_amd import inputs
    return np.stack([inputs.gaussian_bumps_state(om.verts, om.cell_verts, om.edge_verts, nb, s)
                     for s in seeds])


def to_dev(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")
