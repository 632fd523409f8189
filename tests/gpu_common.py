"""Shared set-up of the GPU parity tests: the same seeded inputs on the
oracle's mesh and on the library's mesh, mapped by geometry."""
import functools

import numpy as np

from matching import MeshMap

PARITY = dict(cheb_tol=1e-13, cg_rtol=1e-14)


def rel_w(ops_oracle, a, b):
    return ops_oracle.wnorm(a - b) / ops_oracle.wnorm(b)


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
