"""Oracle: tetrahedral mesh, canonical numbering, incidence matrices, barycentric geometry.

Sec. II-A: the domain is a set of tetrahedra with N_s nodes, N_e edges and N_f faces; the
de Rham sequence on it gives node (0-form), edge (1-form) and face (2-form) unknowns.

Canonical numbering (an interface both implementations follow, each with its own code):
* every tet's four node ids sorted ascending; local vertex k is the k-th smallest;
* edges = unique sorted node pairs, in lexicographic order; oriented low -> high id;
* faces = unique sorted node triples, in lexicographic order; oriented by the right-hand
  normal (r_j - r_i) x (r_k - r_i) for i < j < k;
* local face k of a tet is the face opposite local vertex k.

Incidence (the exterior derivative on this complex):
* D  [N_e x N_s]: -1 at the tail, +1 at the head of each edge (discrete gradient);
* C  [N_f x N_e]: face (i,j,k) -> +1 (i,j), +1 (j,k), -1 (i,k) (discrete curl; Sec. II-A
  notes that the curl matrix of the Whitney edge functions is this +-1 incidence);
* D2 [N_t x N_f]: (-1)^k on the face opposite local vertex k (discrete divergence).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

LOCAL_EDGES = np.array([(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)], dtype=np.int64)
LOCAL_FACES = np.array([(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)], dtype=np.int64)


def _unique_rows(rows, n_nodes):
    """Unique rows of non-negative ids below n_nodes in lexicographic order, and each
    input row's index among them.  A row (a, b[, c]) is the base-n_nodes number
    a n^2 + b n + c, whose numeric order is the rows' lexicographic order, so a 1-D unique
    of these numbers gives the same result as a unique over rows, faster."""
    rows = np.asarray(rows, dtype=np.int64)
    if float(n_nodes) ** rows.shape[1] >= 2.0 ** 62:
        return np.unique(rows, axis=0, return_inverse=True)
    key = rows[:, 0].copy()
    for j in range(1, rows.shape[1]):
        key = key * n_nodes + rows[:, j]
    u, inv = np.unique(key, return_inverse=True)
    out = np.empty((len(u), rows.shape[1]), dtype=np.int64)
    for j in range(rows.shape[1] - 1, -1, -1):
        out[:, j] = u % n_nodes
        u = u // n_nodes
    return out, inv.reshape(-1)


class Mesh:
    def __init__(self, xyz, tets):
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tets = np.ascontiguousarray(np.sort(np.asarray(tets, dtype=np.int64), axis=1))
        self.n_nodes = self.xyz.shape[0]
        self.n_tets = self.tets.shape[0]
        nt = self.n_tets

        # ---- edges
        inst = self.tets[:, LOCAL_EDGES].reshape(-1, 2)
        self.edges, inv = _unique_rows(inst, self.n_nodes)
        self.tet_edges = inv.reshape(nt, 6).astype(np.int64)
        self.n_edges = self.edges.shape[0]

        # ---- faces
        inst = self.tets[:, LOCAL_FACES].reshape(-1, 3)
        self.faces, inv = _unique_rows(inst, self.n_nodes)
        inv = inv.reshape(-1)
        self.tet_faces = inv.reshape(nt, 4).astype(np.int64)
        self.n_faces = self.faces.shape[0]
        count = np.bincount(inv, minlength=self.n_faces)
        if np.any(count > 2):
            raise ValueError("non-conforming mesh: a face is shared by more than two tets")
        self.boundary_face = count == 1

        # neighbour across the face opposite local vertex k (-1 on the boundary)
        owner = np.repeat(np.arange(nt), 4)
        order = np.argsort(inv, kind="stable")
        f_sorted = inv[order]
        first = np.ones(len(order), dtype=bool)
        first[1:] = f_sorted[1:] != f_sorted[:-1]
        face_tets = -np.ones((self.n_faces, 2), dtype=np.int64)
        face_tets[f_sorted[first], 0] = owner[order[first]]
        second = ~first
        face_tets[f_sorted[second], 1] = owner[order[second]]
        self.face_tets = face_tets
        nbr = -np.ones((nt, 4), dtype=np.int64)
        for k in range(4):
            f = self.tet_faces[:, k]
            a, b = face_tets[f, 0], face_tets[f, 1]
            me = np.arange(nt)
            nbr[:, k] = np.where(a == me, b, a)
        self.nbr = nbr

        # ---- boundary entities
        bf = self.faces[self.boundary_face]
        self.boundary_node = np.zeros(self.n_nodes, dtype=bool)
        self.boundary_node[bf.ravel()] = True
        be = np.concatenate([bf[:, [0, 1]], bf[:, [1, 2]], bf[:, [0, 2]]], axis=0)
        self.boundary_edge = np.zeros(self.n_edges, dtype=bool)
        self.boundary_edge[self.edge_index(be[:, 0], be[:, 1])] = True
        self.interior_edges = np.nonzero(~self.boundary_edge)[0]
        self.interior_nodes = np.nonzero(~self.boundary_node)[0]

        # face -> its three edges, in the order (i,j), (j,k), (i,k)
        f = self.faces
        self.face_edges = np.stack([self.edge_index(f[:, 0], f[:, 1]),
                                    self.edge_index(f[:, 1], f[:, 2]),
                                    self.edge_index(f[:, 0], f[:, 2])], axis=1)

        self._geometry()

    # ------------------------------------------------------------------ lookups
    def edge_index(self, a, b):
        """Index of edge (a,b), a < b, by binary search in the lexicographic edge list."""
        key = self.edges[:, 0] * self.n_nodes + self.edges[:, 1]
        q = np.asarray(a, dtype=np.int64) * self.n_nodes + np.asarray(b, dtype=np.int64)
        idx = np.searchsorted(key, q)
        if np.any(idx >= len(key)) or np.any(key[np.minimum(idx, len(key) - 1)] != q):
            raise KeyError("edge not in mesh")
        return idx

    def euler_characteristic(self):
        return self.n_nodes - self.n_edges + self.n_faces - self.n_tets

    # ------------------------------------------------------------------ incidence
    def D(self):
        ne = self.n_edges
        rows = np.repeat(np.arange(ne), 2)
        cols = self.edges.ravel()
        vals = np.tile([-1.0, 1.0], ne)
        return sp.csr_matrix((vals, (rows, cols)), shape=(ne, self.n_nodes))

    def C(self):
        nf = self.n_faces
        rows = np.repeat(np.arange(nf), 3)
        cols = self.face_edges.ravel()
        vals = np.tile([1.0, 1.0, -1.0], nf)
        return sp.csr_matrix((vals, (rows, cols)), shape=(nf, self.n_edges))

    def D2(self):
        nt = self.n_tets
        rows = np.repeat(np.arange(nt), 4)
        cols = self.tet_faces.ravel()
        vals = np.tile([1.0, -1.0, 1.0, -1.0], nt)
        return sp.csr_matrix((vals, (rows, cols)), shape=(nt, self.n_faces))

    # ------------------------------------------------------------------ geometry
    def _geometry(self):
        """Barycentric coordinate k of tet t is the ratio of signed volumes
        lambda_k(x) = [(x - r_a) . ((r_b - r_a) x (r_c - r_a))] /
                      [(r_k - r_a) . ((r_b - r_a) x (r_c - r_a))],  {a,b,c} = the other three,
        so grad lambda_k = ((r_b - r_a) x (r_c - r_a)) / [(r_k - r_a) . (...)]."""
        r = self.xyz[self.tets]                      # [nt, 4, 3]
        grad = np.empty((self.n_tets, 4, 3))
        for k in range(4):
            a, b, c = LOCAL_FACES[k]
            nrm = np.cross(r[:, b] - r[:, a], r[:, c] - r[:, a])
            den = np.einsum("ij,ij->i", r[:, k] - r[:, a], nrm)
            grad[:, k] = nrm / den[:, None]
        self.grad_lambda = grad
        d = np.einsum("ij,ij->i", r[:, 1] - r[:, 0], np.cross(r[:, 2] - r[:, 0], r[:, 3] - r[:, 0]))
        self.signed_vol6 = d
        self.vol = np.abs(d) / 6.0
        if np.any(self.vol <= 1e-14 * np.max(self.vol)):
            raise ValueError("degenerate tetrahedron")

    def barycentric(self, t, x):
        """lambda_k(x) in tet t (vectorised over rows)."""
        t = np.asarray(t)
        x = np.asarray(x, dtype=np.float64)
        lam = np.empty(x.shape[:-1] + (4,))
        for k in range(4):
            a = LOCAL_FACES[k][0]
            lam[..., k] = np.einsum("...j,...j->...", x - self.xyz[self.tets[t, a]], self.grad_lambda[t, k])
        return lam

    def locate(self, x, n_candidates=48):
        """Tet containing each point: among the tets with the nearest centroids, the one
        whose smallest barycentric coordinate is largest, accepted if >= -1e-12.
        Returns int64 tet ids (-1 if outside the mesh)."""
        x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
        if len(x) > 65536:
            return np.concatenate([self.locate(x[i:i + 65536], n_candidates)
                                   for i in range(0, len(x), 65536)])
        if not hasattr(self, "_kdtree"):
            self._centroid = self.xyz[self.tets].mean(axis=1)
            self._kdtree = cKDTree(self._centroid)
        k = min(n_candidates, self.n_tets)
        _, cand = self._kdtree.query(x, k=k, workers=-1)
        cand = np.asarray(cand).reshape(len(x), k)
        lam = self.barycentric(cand, np.repeat(x[:, None, :], k, axis=1))
        score = lam.min(axis=2)
        best = np.argmax(score, axis=1)
        out = cand[np.arange(len(x)), best]
        out[score[np.arange(len(x)), best] < -1e-12] = -1
        out[~np.all(np.isfinite(x), axis=1)] = -1
        return out.astype(np.int64)

    # ------------------------------------------------------------------ interpolants
    def edge_dofs_of_uniform_field(self, E0):
        """e_ab = integral of the constant field E0 along edge a->b = E0 . (r_b - r_a)."""
        d = self.xyz[self.edges[:, 1]] - self.xyz[self.edges[:, 0]]
        return d @ np.asarray(E0, dtype=np.float64)

    def face_area_vectors(self):
        f = self.faces
        r = self.xyz
        return 0.5 * np.cross(r[f[:, 1]] - r[f[:, 0]], r[f[:, 2]] - r[f[:, 0]])

    def face_dofs_of_uniform_field(self, B0):
        """b_f = flux of the constant field B0 through face f = B0 . area vector."""
        return self.face_area_vectors() @ np.asarray(B0, dtype=np.float64)
