"""Oracle: the paper's own pair of spaces (Sec. 2.5), BDM2 velocity and
P1DG depth, for the linear operator L of eq. ueq_int and the depth equation
after it, on the icosahedral mesh of flat triangles.
TEST INFRASTRUCTURE ONLY: loaded by tests/ (never by the library).

Spaces, per triangle T (in the triangle's own plane, orthonormal frame
e1, e2 with e1 x e2 the outward normal k):
  BDM2: all quadratic tangent vector fields (dimension 12) whose normal
        component is continuous across edges.  Degrees of freedom: the
        normal component u . n_T at the three Gauss-Legendre points of each
        edge (n_T the outward unit normal of T in its plane; the global
        value is the flux density across the edge in its global direction,
        from the edge's first cell to its second, so the two cells carry it
        with opposite signs), and three interior moments, the integrals of
        u . e1, u . e2 and u . (x - x_T)^perp over T (the lowest-order
        Nedelec field space, the standard interior moments of BDM2).
  P1DG: the barycentric coordinates of T.
Operators (eq. ueq_int and the depth equation):
  M_u[i, j] = int phi_i . phi_j,   F[i, j] = int phi_i . (f k x phi_j),
  B[i, q] = int div(phi_i) psi_q,  M_h[q, r] = int psi_q psi_r,
  L(u, eta) = (M_u^-1 (-F u + g B eta), M_h^-1 (-H B^T u)),
with f = 2 Omega z / |x| at the quadrature points and every integral by a
collapsed (Duffy) Gauss-Legendre rule of 5 x 5 points per triangle (exact
for polynomials of degree 8).  Also: exp(t L) by the Chebyshev recurrence
(Sec. 2.4) and the nonlinearity N of Sec. 2.5 on this pair (BDM2P1DG.expL,
BDM2P1DG.nonlinear).  Written with numpy and scipy.sparse in the order
above; no code is shared with the library.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

_GL3 = 0.5 + 0.5 * np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])  # Gauss points on [0, 1]


def _duffy(n=5):
    """Barycentric points (l0, l1, l2) and weights (summing to 1) of the
    collapsed Gauss-Legendre rule on the reference triangle."""
    x, w = np.polynomial.legendre.leggauss(n)
    x, w = 0.5 * (x + 1.0), 0.5 * w
    a, b = np.meshgrid(x, x, indexing="ij")
    wa, wb = np.meshgrid(w, w, indexing="ij")
    l1 = a.ravel()
    l2 = (b * (1.0 - a)).ravel()
    wt = (wa * wb * (1.0 - a)).ravel() * 2.0  # reference area 1/2 -> weights sum to 1
    return np.stack([1.0 - l1 - l2, l1, l2], axis=1), wt


def _p2(l):
    """The six quadratic Lagrange functions of barycentric points l [..., 3]
    and their derivatives with respect to (l0, l1, l2)."""
    l0, l1, l2 = l[..., 0], l[..., 1], l[..., 2]
    N = np.stack([l0 * (2 * l0 - 1), l1 * (2 * l1 - 1), l2 * (2 * l2 - 1),
                  4 * l1 * l2, 4 * l0 * l2, 4 * l0 * l1], axis=-1)
    z = np.zeros_like(l0)
    dN = np.stack([
        np.stack([4 * l0 - 1, z, z], -1), np.stack([z, 4 * l1 - 1, z], -1),
        np.stack([z, z, 4 * l2 - 1], -1), np.stack([z, 4 * l2, 4 * l1], -1),
        np.stack([4 * l2, z, 4 * l0], -1), np.stack([4 * l1, 4 * l0, z], -1)], axis=-2)
    return N, dN  # [..., 6], [..., 6, 3]


class BDM2P1DG:
    """BDM2 x P1DG operators of the linear shallow-water operator on an
    oracle mesh (oracle.Mesh)."""

    def __init__(self, mesh, g=9.80616, H=1000.0, Omega=7.292e-5):
        self.mesh, self.g, self.H, self.Omega = mesh, g, H, Omega
        V = np.asarray(mesh.verts)
        tri = np.asarray(mesh.cell_verts)
        ce = np.asarray(mesh.cell_edges)
        cs = np.asarray(mesh.cell_sign)
        ev = np.asarray(mesh.edge_verts)
        ne, nc = mesh.ne, mesh.nc
        self.nu, self.nh = 3 * ne + 3 * nc, 3 * nc
        P = V[tri]                                   # [nc, 3, 3]
        e1 = P[:, 1] - P[:, 0]
        e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
        k = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
        area = 0.5 * np.linalg.norm(k, axis=1)
        k /= np.linalg.norm(k, axis=1, keepdims=True)
        e2 = np.cross(k, e1)
        loc = np.stack([np.einsum("cvd,cd->cv", P - P[:, :1], e) for e in (e1, e2)], -1)  # [nc,3,2]
        # barycentric gradients in the local frame: grad l_i = k x (p_{i+2} - p_{i+1}) / 2A
        gl = np.zeros((nc, 3, 2))
        for i in range(3):
            d = loc[:, (i + 2) % 3] - loc[:, (i + 1) % 3]
            gl[:, i] = np.stack([-d[:, 1], d[:, 0]], -1) / (2.0 * area[:, None])
        self.area = area

        def vec_basis(l):
            """The 12 monomial-Lagrange vector fields N_a e_c at barycentric
            points l [q, 3], per cell: values [nc, q, 12, 2], divergence
            [nc, q, 12]."""
            N, dN = _p2(l)
            q = l.shape[0]
            val = np.zeros((nc, q, 12, 2))
            div = np.zeros((nc, q, 12))
            grad = np.einsum("qaj,cjd->cqad", dN, gl)  # d N_a / d x_d
            for a in range(6):
                for c in range(2):
                    val[:, :, 2 * a + c, c] = N[None, :, a]
                    div[:, :, 2 * a + c] = grad[:, :, a, c]
            return val, div

        # degrees of freedom of the 12 monomial fields -> local dual basis
        A = np.zeros((nc, 12, 12))
        self._n3 = np.zeros((nc, 3, 3))  # outward unit normal of each local edge, 3D
        for i in range(3):  # local edge i: opposite vertex i, global edge ce[:, i]
            e = ce[:, i]
            a_glob, b_glob = ev[e, 0], ev[e, 1]
            # barycentric coordinates of the global a and b vertices in the cell
            la = (tri == a_glob[:, None]).astype(float)
            lb = (tri == b_glob[:, None]).astype(float)
            # outward unit normal of edge i in the cell's plane
            d = loc[:, (i + 2) % 3] - loc[:, (i + 1) % 3]
            n = np.stack([d[:, 1], -d[:, 0]], -1)
            mid = 0.5 * (loc[:, (i + 1) % 3] + loc[:, (i + 2) % 3])
            cen = loc.mean(axis=1)
            flip = np.einsum("cd,cd->c", n, mid - cen) < 0
            n[flip] *= -1.0
            n /= np.linalg.norm(n, axis=1, keepdims=True)
            self._n3[:, i] = n[:, :1] * e1 + n[:, 1:] * e2
            for kq, t in enumerate(_GL3):
                lq = (1.0 - t) * la + t * lb        # [nc, 3]
                N, _ = _p2(lq)
                for a in range(6):
                    for c in range(2):
                        A[:, 3 * i + kq, 2 * a + c] = N[:, a] * n[:, c]
        lq, wq = _duffy(5)
        val, div = vec_basis(lq)
        xq = np.einsum("qv,cvd->cqd", lq, loc)               # local coordinates
        xc = loc.mean(axis=1)
        perp = np.stack([-(xq[..., 1] - xc[:, None, 1]), xq[..., 0] - xc[:, None, 0]], -1)
        wA = wq[None, :] * area[:, None]                      # [nc, q]
        A[:, 9] = np.einsum("cq,cqf->cf", wA, val[..., 0]) / area[:, None]
        A[:, 10] = np.einsum("cq,cqf->cf", wA, val[..., 1]) / area[:, None]
        A[:, 11] = np.einsum("cq,cqfd,cqd->cf", wA, val, perp) / area[:, None] ** 1.5
        self._frame = (P, e1, e2, area, lq, wq, perp)
        C = np.linalg.inv(A)                                  # columns: dual basis
        self._C, self._gl, self._k3 = C, gl, k
        phi = np.einsum("cqfd,cfj->cqjd", val, C)             # [nc, q, 12, 2]
        dphi = np.einsum("cqf,cfj->cqj", div, C)
        # physical quadrature points and Coriolis parameter
        X3 = np.einsum("qv,cvd->cqd", lq, P)
        f = 2.0 * Omega * X3[..., 2] / np.linalg.norm(X3, axis=2)
        phip = np.stack([-phi[..., 1], phi[..., 0]], -1)      # k x phi in the local frame
        Mloc = np.einsum("cq,cqid,cqjd->cij", wA, phi, phi)
        Floc = np.einsum("cq,cq,cqid,cqjd->cij", wA, f, phi, phip)
        Bloc = np.einsum("cq,cqi,qr->cir", wA, dphi, lq)
        # global numbering and signs of the local velocity dofs
        gid = np.zeros((nc, 12), dtype=np.int64)
        sg = np.ones((nc, 12))
        for i in range(3):
            for kq in range(3):
                gid[:, 3 * i + kq] = 3 * ce[:, i] + kq
                sg[:, 3 * i + kq] = cs[:, i]
        for m in range(3):
            gid[:, 9 + m] = 3 * ne + 3 * np.arange(nc) + m
        hid = 3 * np.arange(nc)[:, None] + np.arange(3)[None, :]
        self._gid, self._sg = gid, sg
        S = sg[:, :, None] * sg[:, None, :]

        def asm(loc_, rows, cols, shape):
            r = np.broadcast_to(rows[:, :, None], loc_.shape).ravel()
            c = np.broadcast_to(cols[:, None, :], loc_.shape).ravel()
            return sp.csr_matrix((loc_.ravel(), (r, c)), shape=shape)

        self.Mu = asm(Mloc * S, gid, gid, (self.nu, self.nu))
        self.F = asm(Floc * S, gid, gid, (self.nu, self.nu))
        self.B = asm(Bloc * sg[:, :, None], gid, hid, (self.nu, self.nh))
        Mh = area[:, None, None] * (np.ones((3, 3)) + np.eye(3))[None] / 12.0
        self.Mh = asm(Mh, hid, hid, (self.nh, self.nh))
        self._Mu_lu = spl.splu(self.Mu.tocsc())
        self._Mh_lu = spl.splu(self.Mh.tocsc())
        self.n = self.nu + self.nh

    def apply_L(self, U):
        u, eta = U[:self.nu], U[self.nu:]
        u1 = self._Mu_lu.solve(-(self.F @ u) + self.g * (self.B @ eta))
        e1 = self._Mh_lu.solve(-self.H * (self.B.T @ u))
        return np.concatenate([u1, e1])

    def W(self):
        """Energy inner product blkdiag(H M_u, g M_h), in which L is skew."""
        return sp.block_diag([self.H * self.Mu, self.g * self.Mh]).tocsr()

    def WL(self):
        """W L = blkdiag(H, g) [[-F, g B], [-H B^T, 0]] (no solves)."""
        return sp.bmat([[-self.H * self.F, self.g * self.H * self.B],
                        [-self.g * self.H * self.B.T, None]]).tocsr()

    def _winv(self, x):
        return np.concatenate([self._Mu_lu.solve(x[:self.nu]) / self.H,
                               self._Mh_lu.solve(x[self.nu:]) / self.g])

    def rho(self, tol=1e-12):
        """Spectral radius of L (eigenvalues +-i rho): the largest
        eigenvalue rho^2 of the symmetric generalized problem
        (W L)^T W^-1 (W L) x = rho^2 W x (= -L^2 in the W inner product),
        by Lanczos (ARPACK)."""
        WL = self.WL()
        A = spl.LinearOperator((self.n, self.n), dtype=float,
                               matvec=lambda x: -(WL @ self._winv(WL @ x)))
        Minv = spl.LinearOperator((self.n, self.n), matvec=self._winv, dtype=float)
        vals = spl.eigsh(A, k=1, M=self.W(), Minv=Minv, which="LA", tol=tol,
                         return_eigenvectors=False)
        return float(np.sqrt(vals.max()))

    def interpolate(self, field):
        """BDM2 coefficients of a tangent field given as a function of 3D
        points (returning 3D vectors): the flux density across each edge at
        its Gauss points, measured in the edge's first cell, and the
        interior moments of the field's part in each cell's plane."""
        m = self.mesh
        V = np.asarray(m.verts)
        ev = np.asarray(m.edge_verts)
        ec = np.asarray(m.edge_cells)
        ce = np.asarray(m.cell_edges)
        P, e1, e2, area, lq, wq, perp = self._frame
        u = np.zeros(self.nu)
        # the edge's first cell and the local index of the edge in it
        c0 = ec[:, 0]
        li = np.argmax(ce[c0] == np.arange(m.ne)[:, None], axis=1)
        n0 = self._n3[c0, li]
        for kq, t in enumerate(_GL3):
            x = (1.0 - t) * V[ev[:, 0]] + t * V[ev[:, 1]]
            u[3 * np.arange(m.ne) + kq] = np.einsum("ed,ed->e", field(x), n0)
        X3 = np.einsum("qv,cvd->cqd", lq, P)
        F3 = field(X3.reshape(-1, 3)).reshape(X3.shape)
        f1 = np.einsum("cqd,cd->cq", F3, e1)
        f2 = np.einsum("cqd,cd->cq", F3, e2)
        wA = wq[None, :] * area[:, None]
        base = 3 * m.ne + 3 * np.arange(m.nc)
        u[base] = np.einsum("cq,cq->c", wA, f1) / area
        u[base + 1] = np.einsum("cq,cq->c", wA, f2) / area
        u[base + 2] = np.einsum("cq,cq->c", wA, f1 * perp[..., 0] + f2 * perp[..., 1]) / area ** 1.5
        return u

    def frequency_near(self, omega, iters=30):
        """The frequency of L nearest omega: inverse iteration with the
        shift i omega on (W L - i omega W) x = W x_prev, the Rayleigh
        quotient x^H W L x / x^H W x = i omega_h at the end."""
        WL = self.WL().astype(complex)
        W = self.W().astype(complex)
        lu = spl.splu((WL - 1j * omega * W).tocsc())
        x = np.random.default_rng(3).standard_normal(self.n).astype(complex)
        for _ in range(iters):
            x = lu.solve(W @ x)
            x /= np.sqrt(np.real(np.vdot(x, W @ x)))
        mu = np.vdot(x, WL @ x) / np.vdot(x, W @ x)
        return float(np.imag(mu))

    def expL(self, lambda_bar, t, U, tol=1e-13):
        """exp(t L) U by the paper's modified Chebyshev recurrence (Sec. 2.4,
        eq. cheby) in its complex form as printed, Lbar = lambda_bar |t|,
        coefficients by the oracle's discrete cosine transform and
        truncation (om_cheb_coeffs, om_cheb_truncate); every L application
        solves the two mass matrices exactly (sparse LU).  Returns (result,
        degree)."""
        import oracle
        U = np.asarray(U, dtype=float)
        if t == 0.0:
            return U.copy(), 0
        Lbar = lambda_bar * abs(t)
        a = oracle.cheb_coeffs(Lbar, 2 * int(np.ceil(Lbar)) + 64)
        K = oracle.cheb_truncate(a, tol)
        Lc = lambda X: self.apply_L(X.real) + 1j * self.apply_L(X.imag)
        Pm = None
        P = U.astype(complex)
        acc = a[0] * P
        for k in range(K):
            LP = Lc(P)
            nxt = -1j * t * LP / Lbar if k == 0 else 2.0 * t * LP / (1j * Lbar) - Pm
            Pm, P = P, nxt
            acc = acc + a[k + 1] * nxt
        return acc.real, K

    # ------------------------------------------------------------ nonlinearity
    def _basis_at(self, l):
        """Dual basis at per-cell barycentric points l [nc, q, 3]: values
        [nc, q, 12, 2], Jacobians [nc, q, 12, 2 (component), 2 (derivative)]
        in each cell's frame."""
        N, dN = _p2(l)                                        # [nc,q,6], [nc,q,6,3]
        grad = np.einsum("cqaj,cjd->cqad", dN, self._gl)      # [nc,q,6,2]
        nc, q = l.shape[0], l.shape[1]
        val = np.zeros((nc, q, 12, 2))
        jac = np.zeros((nc, q, 12, 2, 2))
        for a in range(6):
            for c in range(2):
                val[:, :, 2 * a + c, c] = N[:, :, a]
                jac[:, :, 2 * a + c, c, :] = grad[:, :, a, :]
        return (np.einsum("cqfd,cfj->cqjd", val, self._C),
                np.einsum("cqfde,cfj->cqjde", jac, self._C))

    def nonlinear(self, U, b=None):
        """N(U) of Sec. 2.5 on this pair: for every test function w in BDM2
        and psi in P1DG,
          int w . u2 = int u . grad^perp(u^perp . w)
                       - int_Gamma [[n^perp (u^perp . w)]] . u~ + int (div w) |u|^2/2,
          int psi eta2 = int grad psi . u (eta - b) - int_Gamma [[psi u]] (eta - b)~,
        with the readings of the lowest-order oracle (om_nonlin.c): the upwind
        value comes from the cell the flow leaves (normal flux out of c0 > 0:
        c0, else c1), the depth facet term carries a minus sign, and (eta -
        b) on a facet is the upwind value.  Here the flux varies along an
        edge, so the upwind side is chosen at every quadrature point.
        Quadrature: the collapsed 5 x 5 rule in the cells (the volume
        integrands have degree 5), 4-point Gauss-Legendre on every side (the
        facet integrands have degree 6 away from a change of upwind side).
        b: bottom height as P1DG coefficients (nh values) or None (flat).
        Both mass matrices are solved exactly (sparse LU)."""
        m = self.mesh
        nc, ne, nu = m.nc, m.ne, self.nu
        U = np.asarray(U, dtype=float)
        coef = self._sg * U[:nu][self._gid]                   # [nc, 12]
        h = U[nu:] - (0.0 if b is None else np.asarray(b, dtype=float))
        h = h.reshape(nc, 3)
        P, e1, e2, area, lq, wq, perp = self._frame
        wA = wq[None, :] * area[:, None]
        gl = self._gl                                         # [nc, 3, 2]
        # ---- cell integrals
        phi, jac = self._basis_at(np.broadcast_to(lq, (nc,) + lq.shape))
        u = np.einsum("cj,cqjd->cqd", coef, phi)              # [nc, q, 2]
        Ju = np.einsum("cj,cqjde->cqde", coef, jac)           # [nc, q, comp, deriv]
        up = np.stack([-u[..., 1], u[..., 0]], -1)            # k x u
        Jup = np.stack([-Ju[..., 1, :], Ju[..., 0, :]], -2)
        # grad (u^perp . phi_i) = (grad u^perp)^T phi_i + (grad phi_i)^T u^perp
        gq = np.einsum("cqed,cqie->cqid", Jup, phi) + np.einsum("cqe,cqied->cqid", up, jac)
        gq_perp = np.stack([-gq[..., 1], gq[..., 0]], -1)     # k x grad
        divphi = jac[..., 0, 0] + jac[..., 1, 1]              # [nc, q, 12]
        ke = 0.5 * np.einsum("cqd,cqd->cq", u, u)
        rl = (np.einsum("cq,cqd,cqid->ci", wA, u, gq_perp)
              + np.einsum("cq,cqi,cq->ci", wA, divphi, ke))
        hq = np.einsum("cr,qr->cq", h, lq)
        rh = np.einsum("cq,crd,cqd,cq->cr", wA, gl, u, hq)
        # ---- facet integrals: traces at 4 Gauss points of every side, the
        # points ordered from the edge's first vertex to its second
        x4, w4 = np.polynomial.legendre.leggauss(4)
        t4, w4 = 0.5 * (x4 + 1.0), 0.5 * w4
        tri = np.asarray(m.cell_verts)
        ce = np.asarray(m.cell_edges)
        ev = np.asarray(m.edge_verts)
        ec = np.asarray(m.edge_cells)
        lf = np.zeros((nc, 3, 4, 3))
        for i in range(3):
            la = (tri == ev[ce[:, i], 0][:, None]).astype(float)
            lb = (tri == ev[ce[:, i], 1][:, None]).astype(float)
            lf[:, i] = (1.0 - t4)[None, :, None] * la[:, None] + t4[None, :, None] * lb[:, None]
        phf, _ = self._basis_at(lf.reshape(nc, 12, 3))
        phf = phf.reshape(nc, 3, 4, 12, 2)
        uf = np.einsum("cj,cspjd->cspd", coef, phf)           # own trace [nc, 3, 4, 2]
        nloc = np.einsum("csd,cd->cs", self._n3, e1), np.einsum("csd,cd->cs", self._n3, e2)
        nloc = np.stack(nloc, -1)                             # outward normals [nc, 3, 2]
        flux = np.einsum("cspd,csd->csp", uf, nloc)           # u . n_out
        uf3 = uf[..., :1] * e1[:, None, None] + uf[..., 1:] * e2[:, None, None]
        hf = np.einsum("cr,cspr->csp", h, lf)
        # upwind cell per edge point: from c0's trace of the flux
        side = np.argmax(ce[ec] == np.arange(ne)[:, None, None], axis=2)   # [ne, 2]
        f0 = flux[ec[:, 0], side[:, 0]]                       # [ne, 4]
        pick = np.where(f0 > 0, 0, 1)                         # 0: c0, 1: c1
        cu = np.take_along_axis(ec, pick, 1)
        su = np.take_along_axis(side, pick, 1)
        ut = uf3[cu, su, np.arange(4)[None, :]]               # [ne, 4, 3]
        ht = hf[cu, su, np.arange(4)[None, :]]                # [ne, 4]
        # side lengths (edge i joins the cell's vertices i+1, i+2)
        lens = np.stack([np.linalg.norm(P[:, (i + 2) % 3] - P[:, (i + 1) % 3], axis=1)
                         for i in range(3)], 1)               # [nc, 3]
        wl = lens[:, :, None] * w4[None, None, :]             # [nc, 3, 4]
        n3 = self._n3                                         # [nc, 3, 3]
        nperp3 = np.cross(self._k3[:, None, :], n3)           # k x n_out
        utc, htc = ut[ce], ht[ce]                             # upwind values seen by each cell side
        upf = np.stack([-uf[..., 1], uf[..., 0]], -1)         # own u^perp
        qf = np.einsum("cspd,cspid->cspi", upf, phf)          # u^perp . phi_i
        rl -= np.einsum("csp,csd,cspd,cspi->ci", wl, nperp3, utc, qf)
        rh -= np.einsum("csp,cspr,csp,csp->cr", wl, lf, flux, htc)
        # ---- assemble and solve
        rhs_u = np.zeros(nu)
        np.add.at(rhs_u, self._gid.ravel(), (self._sg * rl).ravel())
        u2 = self._Mu_lu.solve(rhs_u)
        e2_ = self._Mh_lu.solve(rh.ravel())
        return np.concatenate([u2, e2_])


    # ------------------------------------------------------ averaged rhs
    def phase_avg_rhs(self, lambda_bar, s, w, U, inner="N", tol=1e-13, b=None):
        """Nbar(U) = sum_m w_m exp(-s_m L) N(exp(s_m L) U), eq. vt_discretised
        of Sec. 2.2, every exponential by expL (Sec. 2.4) and N by nonlinear
        (Sec. 2.5, over the bottom b, P1DG coefficients or None); inner =
        "L" or "I" substitutes L or the identity for N (the averages then
        reduce to L U and U)."""
        f = {"N": lambda X: self.nonlinear(X, b=b), "L": self.apply_L,
             "I": lambda X: np.array(X, copy=True)}[inner]
        out = np.zeros(self.n)
        for sm, wm in zip(s, w):
            V, _ = self.expL(lambda_bar, sm, U, tol)
            Y, _ = self.expL(lambda_bar, -sm, f(V), tol)
            out += wm * Y
        return out

    # ------------------------------------------------------------ RK4 step
    def step(self, lambda_bar, s, w, dt, U, inner="N", tol=1e-13, b=None):
        """One step of the averaged system (Sec. 2.3): the Lawson form of
        the classical fourth-order Runge-Kutta method on the averaged
        equation, with the stages in the paper's order (stages 2 and 4 take
        exp(L dt/2) inside N, after exp(L s)), every exponential by expL and
        the averages by phase_avg_rhs (inner and the bottom b as there)."""
        U = np.asarray(U, dtype=float)
        E = lambda t, X: self.expL(lambda_bar, t, X, tol)[0]  # noqa: E731
        f = {"N": lambda X: self.nonlinear(X, b=b), "L": self.apply_L,
             "I": lambda X: np.array(X, copy=True)}[inner]
        h = 0.5 * dt

        def shifted(X):  # sum_m w_m exp(-s_m L) N(exp(L dt/2) exp(s_m L) X)
            out = np.zeros(self.n)
            for sm, wm in zip(s, w):
                out += wm * E(-sm, f(E(h, E(sm, X))))
            return out
        k1 = self.phase_avg_rhs(lambda_bar, s, w, U, inner, tol, b)
        U1 = U + h * k1
        Eh = E(h, U)
        k2 = shifted(U1)
        U2 = Eh + h * k2
        k3 = self.phase_avg_rhs(lambda_bar, s, w, U2, inner, tol, b)
        U3 = Eh + dt * k3
        k4 = shifted(U3)
        return (E(dt, U) + dt / 6.0 * (E(dt, k1) + 2.0 * E(h, k2) + 2.0 * E(h, k3) + k4))
