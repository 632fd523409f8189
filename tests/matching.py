"""Map states between two independently numbered copies of the same mesh by
geometry: cells by centroid, edges by midpoint, edge signs by the direction
of the a -> b traversal (which fixes the direction of the edge normal)."""
import numpy as np
from scipy.spatial import cKDTree


class MeshMap:
    def __init__(self, src, dst):
        """src, dst: objects with verts, cell_verts, edge_verts arrays."""
        cs = src.verts[src.cell_verts].mean(axis=1)
        cd = dst.verts[dst.cell_verts].mean(axis=1)
        d, self.cell = cKDTree(cs).query(cd)  # dst cell i <- src cell self.cell[i]
        assert d.max() < 1e-6 * np.linalg.norm(cs, axis=1).max()
        ms = 0.5 * (src.verts[src.edge_verts[:, 0]] + src.verts[src.edge_verts[:, 1]])
        md = 0.5 * (dst.verts[dst.edge_verts[:, 0]] + dst.verts[dst.edge_verts[:, 1]])
        d, self.edge = cKDTree(ms).query(md)
        assert d.max() < 1e-6 * np.linalg.norm(ms, axis=1).max()
        ts = src.verts[src.edge_verts[:, 1]] - src.verts[src.edge_verts[:, 0]]
        td = dst.verts[dst.edge_verts[:, 1]] - dst.verts[dst.edge_verts[:, 0]]
        dots = np.einsum("ij,ij->i", ts[self.edge], td)
        self.sign = np.sign(dots)
        assert np.all(np.abs(dots) > 0.5 * np.einsum("ij,ij->i", td, td))
        self.ne_src = len(src.edge_verts)
        self.ne = len(dst.edge_verts)
        assert len(np.unique(self.cell)) == len(self.cell)
        assert len(np.unique(self.edge)) == len(self.edge)

    def state(self, U):
        """src state(s) [..., n] -> dst numbering."""
        U = np.asarray(U)
        u = U[..., :self.ne_src][..., self.edge] * self.sign
        eta = U[..., self.ne_src:][..., self.cell]
        return np.concatenate([u, eta], axis=-1)

    def back(self, V):
        """dst state(s) [..., n] -> src numbering."""
        V = np.asarray(V)
        u = np.zeros(V.shape[:-1] + (self.ne_src,))
        u[..., self.edge] = V[..., :self.ne] * self.sign
        eta = np.zeros(V.shape[:-1] + (len(self.cell),))
        eta[..., self.cell] = V[..., self.ne:]
        return np.concatenate([u, eta], axis=-1)
