"""Reference of the learned mass-matrix preconditioner, plain numpy in FP64.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline use it; the library never does.

The paper solves its velocity mass systems by preconditioned conjugate
gradients (end of Sec. 2.5); a learned preconditioner is not part of the
paper.  This module is the complete definition that the GPU implementation
follows, written out step by step with manual backpropagation and no
blocking or fusion:

Features (all dimensionless; every quantity is invariant under renumbering
and under flipping an edge's orientation):
  edge e with cells c0, c1 and endpoints a, b:
    0  M_ee, the diagonal of the velocity mass matrix
    1  |e| / mean edge length
    2  (|c0| + |c1|) / (2 mean cell area)
    3  z/|x| at the edge midpoint (f / 2 Omega)
    4  mean of the cosines of the two angles opposite e (in c0 and in c1)
    5  |difference| of those two cosines
    6  mean of the four cosines of the angles at a and b in c0 and c1
    7  max - min of those four cosines
  cell c:
    0  |c| / mean cell area
    1  z/|x| at the centroid
    2  max - min of the cosines of its three angles
    3  mean of M_ee over its three edges
Network (width 32, relu):
  he = relu(Fe W_ee + b_ee),  hc = relu(Fc W_ce + b_ce)
  three rounds:  hc = relu([hc, mean of he over the 3 edges of c] W_cl + b_cl)
                 he = relu([he, mean of hc over the 2 cells of e] W_el + b_el)
  diagonal head:  g_ii = softplus(he_i . w_hd + b_hd)
  pair head, for each ordered pair (i, j) of distinct edges of a cell c:
                 z = relu([he_i, he_j, hc_c] W_p1 + b_p1),  beta_ij = z . w_p2 + b_p2
  Ghat_ii = g_ii,  Ghat_ij = beta_ij Mhat_ij  with Mhat = D^-1/2 M D^-1/2,
  and the preconditioner P = D^-1/2 Ghat Ghat^T D^-1/2 (symmetric positive
  semi-definite by construction, definite when Ghat is non-singular).
Loss over probe vectors z_p (columns of Z):
  L = (1/P) sum_p |Ghat^T Mhat Ghat z_p - z_p|^2 / |z_p|^2
which is zero exactly when Ghat^T Mhat Ghat = I, i.e. P M = I.
Initial parameters: Glorot-uniform weights from SplitMix64(seed), zero
biases, zero output weights of both heads, b_hd = log(e - 1) and b_p2 = 0,
so that the initial Ghat is the identity and P is the Jacobi preconditioner.

Parity pins (tests/test_oracle_lp.py): central finite differences of the
loss against the manual gradient; the loss with identity probes against
the dense Frobenius norm of Ghat^T Mhat Ghat - I; the initial network gives
Ghat = I; P is positive definite on probes.
"""
import math

import numpy as np

FE, FC, WIDTH, LAYERS = 8, 4, 32, 3


def param_shapes():
    """Names and shapes of the parameters, in storage order (each weight
    matrix is [inputs][outputs], row-major)."""
    W = WIDTH
    s = [("ee.W", (FE, W)), ("ee.b", (W,)), ("ce.W", (FC, W)), ("ce.b", (W,))]
    for l in range(LAYERS):
        s += [(f"cl{l}.W", (2 * W, W)), (f"cl{l}.b", (W,)),
              (f"el{l}.W", (2 * W, W)), (f"el{l}.b", (W,))]
    s += [("hd.w", (W,)), ("hd.b", (1,)), ("p1.W", (3 * W, W)), ("p1.b", (W,)),
          ("p2.w", (W,)), ("p2.b", (1,))]
    return s


def n_params():
    return sum(int(np.prod(sh)) for _, sh in param_shapes())


def unpack(theta):
    out, off = {}, 0
    for name, sh in param_shapes():
        n = int(np.prod(sh))
        out[name] = np.asarray(theta[off:off + n], np.float64).reshape(sh)
        off += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in param_shapes()])


def _splitmix_uniform(seed, n):
    """n uniforms in [0, 1) from SplitMix64 (Steele, Lea and Flood 2014),
    53-bit mantissas."""
    mask = (1 << 64) - 1
    x = seed & mask
    out = np.empty(n)
    for i in range(n):
        x = (x + 0x9E3779B97F4A7C15) & mask
        z = x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        z = z ^ (z >> 31)
        out[i] = (z >> 11) * (1.0 / (1 << 53))
    return out


def init_params(seed):
    """Initial parameters (see the module docstring), drawn in storage order:
    each weight matrix W[k][o] takes the next k*o uniforms u, as
    (2u - 1) sqrt(6 / (fan_in + fan_out)); biases and head outputs take none."""
    d = {}
    draws = []
    for name, sh in param_shapes():
        if name.endswith(".W"):
            draws.append((name, sh))
    total = sum(int(np.prod(sh)) for _, sh in draws)
    u = _splitmix_uniform(seed, total)
    off = 0
    for name, sh in param_shapes():
        if name.endswith(".W"):
            n = int(np.prod(sh))
            lim = math.sqrt(6.0 / (sh[0] + sh[1]))
            d[name] = ((2.0 * u[off:off + n] - 1.0) * lim).reshape(sh)
            off += n
        else:
            d[name] = np.zeros(sh)
    d["hd.b"][:] = math.log(math.e - 1.0)
    return pack(d)


class Graph:
    """Features, adjacency and scaled mass entries of one operator, from the
    oracle mesh and the oracle's assembled mass matrix."""

    def __init__(self, mesh, ops):
        ex = ops.export()
        ne, nc = mesh.ne, mesh.nc
        rows = np.repeat(np.arange(ne), np.diff(ex["rowptr"]))
        Md = {}
        for r, c, v in zip(rows, ex["cols"], ex["mass"]):
            Md[(int(r), int(c))] = Md.get((int(r), int(c)), 0.0) + v
        diag = np.array([Md[(e, e)] for e in range(ne)])
        X = mesh.verts
        cv, ce, ec, ev = mesh.cell_verts, mesh.cell_edges, mesh.edge_cells, mesh.edge_verts
        area = ex["area"]
        self.ne, self.nc = ne, nc
        self.ce, self.ec = ce.astype(np.int64), ec.astype(np.int64)
        self.diag = diag

        def cos_at(c, vert):
            """cosine of the angle of cell c at its vertex `vert`"""
            vs = list(cv[c])
            k = vs.index(vert)
            a, b, d = X[vs[k]], X[vs[(k + 1) % 3]], X[vs[(k + 2) % 3]]
            u, v = b - a, d - a
            return float(u @ v / (np.linalg.norm(u) * np.linalg.norm(v)))

        elen = np.linalg.norm(X[ev[:, 0]] - X[ev[:, 1]], axis=1)
        lbar, abar = elen.mean(), area.mean()
        Fe = np.zeros((ne, FE))
        for e in range(ne):
            a, b = int(ev[e, 0]), int(ev[e, 1])
            opp, ends = [], []
            for c in ec[e]:
                other = [v for v in cv[c] if v != a and v != b][0]
                opp.append(cos_at(c, other))
                ends += [cos_at(c, a), cos_at(c, b)]
            mid = 0.5 * (X[a] + X[b])
            Fe[e] = [diag[e], elen[e] / lbar, (area[ec[e, 0]] + area[ec[e, 1]]) / (2 * abar),
                     mid[2] / np.linalg.norm(mid), 0.5 * (opp[0] + opp[1]), abs(opp[0] - opp[1]),
                     np.mean(ends), max(ends) - min(ends)]
        Fc = np.zeros((nc, FC))
        for c in range(nc):
            cs = [cos_at(c, int(v)) for v in cv[c]]
            cen = X[cv[c]].mean(0)
            Fc[c] = [area[c] / abar, cen[2] / np.linalg.norm(cen), max(cs) - min(cs),
                     np.mean(diag[ce[c]])]
        self.Fe, self.Fc = Fe, Fc
        # ordered pairs (i, j) of distinct edges of a cell, with that cell
        pi, pj, pc = [], [], []
        for c in range(nc):
            for a in range(3):
                for b in range(3):
                    if a != b:
                        pi.append(ce[c, a])
                        pj.append(ce[c, b])
                        pc.append(c)
        self.pi, self.pj, self.pc = (np.array(v, np.int64) for v in (pi, pj, pc))
        self.mhat = np.array([Md[(int(i), int(j))] / math.sqrt(diag[i] * diag[j])
                              for i, j in zip(self.pi, self.pj)])
        # scaled mass matrix as (row, col, value) triplets
        self.m_rows = np.array([k[0] for k in Md], np.int64)
        self.m_cols = np.array([k[1] for k in Md], np.int64)
        self.m_vals = np.array([v / math.sqrt(diag[k[0]] * diag[k[1]]) for k, v in Md.items()])


def _relu(x):
    return np.maximum(x, 0.0)


def _softplus(x):
    return np.logaddexp(0.0, x)


def _sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def forward(theta, g):
    """Activations of every layer and the entries of Ghat: (cache, gdiag,
    beta, goff) with goff = beta * mhat for the ordered pairs of g."""
    p = unpack(theta)
    cache = {}
    he = _relu(g.Fe @ p["ee.W"] + p["ee.b"])
    hc = _relu(g.Fc @ p["ce.W"] + p["ce.b"])
    cache["he0"], cache["hc0"] = he, hc
    for l in range(LAYERS):
        xc = np.concatenate([hc, he[g.ce].mean(axis=1)], axis=1)
        hc = _relu(xc @ p[f"cl{l}.W"] + p[f"cl{l}.b"])
        xe = np.concatenate([he, hc[g.ec].mean(axis=1)], axis=1)
        he = _relu(xe @ p[f"el{l}.W"] + p[f"el{l}.b"])
        cache[f"xc{l}"], cache[f"hc{l + 1}"] = xc, hc
        cache[f"xe{l}"], cache[f"he{l + 1}"] = xe, he
    gam = he @ p["hd.w"] + p["hd.b"][0]
    xp = np.concatenate([he[g.pi], he[g.pj], hc[g.pc]], axis=1)
    z = _relu(xp @ p["p1.W"] + p["p1.b"])
    beta = z @ p["p2.w"] + p["p2.b"][0]
    cache.update(gam=gam, xp=xp, z=z)
    return cache, _softplus(gam), beta, beta * g.mhat


def _apply_G(g, gdiag, goff, v):
    out = gdiag[:, None] * v
    np.add.at(out, g.pi, goff[:, None] * v[g.pj])
    return out


def _apply_GT(g, gdiag, goff, v):
    out = gdiag[:, None] * v
    np.add.at(out, g.pj, goff[:, None] * v[g.pi])
    return out


def _apply_M(g, v):
    out = np.zeros_like(v)
    np.add.at(out, g.m_rows, g.m_vals[:, None] * v[g.m_cols])
    return out


def loss_and_ghat_grad(g, gdiag, goff, Z):
    """L and dL/dGhat (diagonal, pair entries) for probes Z [ne][P]."""
    P = Z.shape[1]
    zz = (Z * Z).sum(axis=0)
    y = _apply_G(g, gdiag, goff, Z)
    w = _apply_M(g, y)
    a = _apply_GT(g, gdiag, goff, w)
    res = a - Z
    L = float(((res * res).sum(axis=0) / zz).sum() / P)
    u = _apply_M(g, _apply_G(g, gdiag, goff, res))
    # dL/dGhat_ij = (2/P) sum_p (w_i res_j + u_i z_j) / |z_p|^2
    s = 2.0 / (P * zz)
    d_diag = ((w * res + u * Z) * s).sum(axis=1)
    d_off = ((w[g.pi] * res[g.pj] + u[g.pi] * Z[g.pj]) * s).sum(axis=1)
    return L, d_diag, d_off


def loss_grad(theta, g, Z):
    """Loss and its gradient with respect to every parameter (manual
    backpropagation through the heads, the three rounds and the encoders)."""
    p = unpack(theta)
    cache, gdiag, beta, goff = forward(theta, g)
    L, d_diag, d_off = loss_and_ghat_grad(g, gdiag, goff, Z)
    gr = {k: np.zeros_like(v) for k, v in p.items()}
    # heads
    dgam = d_diag * _sigmoid(cache["gam"])
    dbeta = d_off * g.mhat
    he, hc = cache[f"he{LAYERS}"], cache[f"hc{LAYERS}"]
    gr["hd.w"] = he.T @ dgam
    gr["hd.b"] = np.array([dgam.sum()])
    dhe = np.outer(dgam, p["hd.w"])
    gr["p2.w"] = cache["z"].T @ dbeta
    gr["p2.b"] = np.array([dbeta.sum()])
    dz = np.outer(dbeta, p["p2.w"]) * (cache["z"] > 0)
    gr["p1.W"] = cache["xp"].T @ dz
    gr["p1.b"] = dz.sum(axis=0)
    dxp = dz @ p["p1.W"].T
    W = WIDTH
    np.add.at(dhe, g.pi, dxp[:, :W])
    np.add.at(dhe, g.pj, dxp[:, W:2 * W])
    dhc = np.zeros_like(hc)
    np.add.at(dhc, g.pc, dxp[:, 2 * W:])
    # rounds, last to first
    for l in reversed(range(LAYERS)):
        dpre = dhe * (cache[f"he{l + 1}"] > 0)
        gr[f"el{l}.W"] = cache[f"xe{l}"].T @ dpre
        gr[f"el{l}.b"] = dpre.sum(axis=0)
        dxe = dpre @ p[f"el{l}.W"].T
        dhe = dxe[:, :W].copy()
        for s in range(2):
            np.add.at(dhc, g.ec[:, s], 0.5 * dxe[:, W:])
        dpre = dhc * (cache[f"hc{l + 1}"] > 0)
        gr[f"cl{l}.W"] = cache[f"xc{l}"].T @ dpre
        gr[f"cl{l}.b"] = dpre.sum(axis=0)
        dxc = dpre @ p[f"cl{l}.W"].T
        dhc = dxc[:, :W].copy()
        for s in range(3):
            np.add.at(dhe, g.ce[:, s], dxc[:, W:] / 3.0)
    dpre = dhe * (cache["he0"] > 0)
    gr["ee.W"] = g.Fe.T @ dpre
    gr["ee.b"] = dpre.sum(axis=0)
    dpre = dhc * (cache["hc0"] > 0)
    gr["ce.W"] = g.Fc.T @ dpre
    gr["ce.b"] = dpre.sum(axis=0)
    return L, pack(gr)


def ghat_dense(g, gdiag, goff):
    G = np.diag(gdiag)
    np.add.at(G, (g.pi, g.pj), goff)
    return G


def mhat_dense(g):
    Mh = np.zeros((g.ne, g.ne))
    np.add.at(Mh, (g.m_rows, g.m_cols), g.m_vals)
    return Mh
